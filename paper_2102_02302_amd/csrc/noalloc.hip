// cleora_propagate_rows_noalloc: cleora_propagate_rows for callers that
// cannot allocate device memory.  Every buffer the call needs beyond its
// inputs and output (the CSR build's sort keys and scan space, the CSR
// itself, the propagation schedule, split-row partial sums, the step
// descriptor and the rows' staging) is carved out of one static device
// array per GPU, sized for the limits in cleora.h.  The kernels are those of
// cleora_propagate_rows; only where their buffers live differs.
#include <mutex>

#include "internal.hpp"

namespace {

using cleora::DevBuf;
using cleora::Error;

constexpr int64_t MAX_ROWS = CLEORA_NOALLOC_MAX_ROWS;
constexpr int64_t MAX_EDGES = CLEORA_NOALLOC_MAX_EDGES;
constexpr int64_t MAX_ROW_BYTES = CLEORA_NOALLOC_MAX_ROW_BYTES;
constexpr int64_t SPLIT = 512;  // the library's split size (no per-call setting here)

size_t al(size_t x) { return (x + 255) / 256 * 256; }

// Bytes of each carved buffer at the limits, following the sizes the CSR
// build and the schedule ask for (directed build: one stored entry per
// edge).  A call never asks for more: a fixed buffer that would need more
// raises E_INVAL instead of allocating.
struct Layout {
    size_t small, keys, tmp, esum, head, cnt, pos, scan, wts, rp, col, val, deg;
    size_t chunk_base, split_items, long_rows, bucket_row, partial, desc, out;
    size_t total() const
    {
        return al(small) + al(keys) + al(tmp) + al(esum) + al(head) + al(cnt) + al(pos) +
               al(scan) + al(wts) + al(rp) + al(col) + al(val) + al(deg) + al(chunk_base) +
               al(split_items) + al(long_rows) + al(bucket_row) + al(partial) + al(desc) +
               al(out);
    }
};

Layout layout_at_limits()
{
    const size_t M = MAX_EDGES, R = MAX_ROWS;
    // radix-sort blocks hold at least 256 keys, so 256 counts per block
    // need at most M + 256 entries
    const size_t nblk = M / 256 + 1, scan_max = std::max(M + 1, 256 * nblk + 1);
    const size_t n_split = 2 * M / SPLIT + 1;  // pieces of rows longer than SPLIT
    Layout L{};
    L.small = 8 * sizeof(int64_t);
    L.keys = 8 * M;
    L.tmp = 8 * M;
    L.esum = 8 * M;
    L.head = M;
    L.cnt = 4 * std::max(256 * nblk, 2 * R);
    L.pos = 8 * scan_max;
    L.scan = 8 * cleora::scan_workspace_elems((int64_t)scan_max);
    L.wts = 8 * M;
    L.rp = 8 * (R + 1);
    L.col = 4 * M;
    L.val = 4 * M;
    L.deg = 8 * R;
    L.chunk_base = 8 * (R + 1);
    L.split_items = 8 * n_split;
    L.long_rows = 4 * (M / SPLIT + 1);
    L.bucket_row = 4 * ((M + R) / 16 + 3);  // packing size >= 16 entries
    // float32 partial rows of ld elements: 4 * ld bytes (ld of a bf16 row
    // is half its bytes)
    L.partial = n_split * 2 * MAX_ROW_BYTES;
    L.desc = 2 * sizeof(cleora::StepDesc);
    L.out = R * MAX_ROW_BYTES;
    return L;
}

constexpr size_t SCRATCH_BYTES = 80ull << 20;  // the layout at the limits is about 77 MB

// The scratch array: one copy on every GPU the library runs on, held until
// the process ends.  In host code its name is a host-side stand-in: only
// the address hipGetSymbolAddress returns (per device) is used.
__device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
unsigned char *g_scratch[MAX_DEVICES] = {};
int64_t g_small[MAX_DEVICES][8] = {};  // host mirror of the build's status words

unsigned char *scratch_on(int device)
{
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[device]) {
        void *p = nullptr;
        CLEORA_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) throw Error(CLEORA_E_DEVICE, "no address for the static scratch array");
        g_scratch[device] = static_cast<unsigned char *>(p);
    }
    return g_scratch[device];
}

void carve(DevBuf &b, unsigned char *&at, size_t bytes)
{
    b.p = at;
    b.cap = bytes;
    b.fixed = true;
    at += al(bytes);
}

}  // namespace

extern "C" int cleora_propagate_rows_noalloc(int device, int64_t n_rows, int64_t n_cols,
                                             int64_t n_edges, const int32_t *rows,
                                             const int32_t *cols, const float *w,
                                             const void *T_in, int64_t ld_in, int32_t dim,
                                             int32_t dtype, void *out, int64_t ld_out,
                                             void *stream)
{
    try {
        cleora::TraceRange trace_range("cleora_propagate_rows_noalloc");
        cleora::check_rows_args(n_rows, n_cols, n_edges, rows, cols, T_in, ld_in, dim, dtype,
                                out, ld_out);
        const int64_t row_bytes = ld_in * (dtype == CLEORA_BF16 ? 2 : 4);
        if (n_rows > MAX_ROWS || n_edges > MAX_EDGES || row_bytes > MAX_ROW_BYTES)
            throw Error(CLEORA_E_INVAL,
                        "above the no-allocation limits (" + std::to_string(MAX_ROWS) +
                            " rows, " + std::to_string(MAX_EDGES) + " edges, " +
                            std::to_string(MAX_ROW_BYTES) + " bytes per row)");
        int count = 0;
        CLEORA_HIP(hipGetDeviceCount(&count));
        if (device < 0 || device >= count || device >= MAX_DEVICES)
            throw Error(CLEORA_E_DEVICE, "no such device");
        int prev = -1;
        CLEORA_HIP(hipGetDevice(&prev));
        if (prev != device) CLEORA_HIP(hipSetDevice(device));
        struct Restore {
            int prev, dev;
            ~Restore()
            {
                if (prev >= 0 && prev != dev) (void)hipSetDevice(prev);
            }
        } restore{prev, device};

        static const Layout L = layout_at_limits();
        if (L.total() > SCRATCH_BYTES) throw Error(CLEORA_E_DEVICE, "scratch layout too large");
        unsigned char *at = scratch_on(device);
        // a context whose buffers are views into the scratch array (no
        // cleora_create: that allocates pinned host memory)
        cleora_ctx c;
        c.device = device;
        c.h_small = g_small[device];
        carve(c.t_small, at, L.small);
        carve(c.t_keys, at, L.keys);
        carve(c.t_tmp, at, L.tmp);
        carve(c.t_esum, at, L.esum);
        carve(c.t_head, at, L.head);
        carve(c.t_cnt, at, L.cnt);
        carve(c.t_pos, at, L.pos);
        carve(c.t_scan, at, L.scan);
        carve(c.t_wts, at, L.wts);
        carve(c.rp, at, L.rp);
        carve(c.col, at, L.col);
        carve(c.val, at, L.val);
        carve(c.deg, at, L.deg);
        carve(c.chunk_base, at, L.chunk_base);
        carve(c.split_items, at, L.split_items);
        carve(c.long_rows, at, L.long_rows);
        carve(c.bucket_row, at, L.bucket_row);
        carve(c.partial, at, L.partial);
        carve(c.desc, at, L.desc);
        carve(c.E[1], at, L.out);
        cleora::propagate_rows_into(&c, n_rows, n_cols, n_edges, rows, cols, w, T_in, dim, dtype,
                                    out, ld_out, cleora::as_stream(stream));
        return CLEORA_OK;
    } catch (const Error &e) {
        cleora::set_last_error(e.what());
        return e.code;
    } catch (const std::bad_alloc &) {
        cleora::set_last_error("host allocation failed");
        return CLEORA_E_NOMEM;
    } catch (const std::exception &e) {
        cleora::set_last_error(e.what());
        return CLEORA_E_DEVICE;
    } catch (...) {
        cleora::set_last_error("unknown error");
        return CLEORA_E_DEVICE;
    }
}
