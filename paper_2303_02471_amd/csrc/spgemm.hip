// Host side of the C ABI (include/spgemm.h): argument checks, plans, device
// workspace, and the launch sequence of every phase.
//
// Symbolic:  classify (Op_j, accumulator bin) -> place (bin lists) ->
//            product-space offsets -> expansion (row of every product) ->
//            ESC / workgroup accumulators: distinct rows per column and the
//            destination of every product -> prefix scan into the column
//            pointers -> one device-to-host copy of the totals.
// Numeric:   every product formed and written or staged through its
//            destination, then the staged later products added in order.
// Backward:  row view of B (once per plan) -> sampled products for dB, dA.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <mutex>
#include <new>
#include <optional>
#include <vector>

#include "../../include/spgemm.h"
#include "internal.h"

using namespace spg;

// Device memory of a plan, from the allocator the plan was created with: the
// caller's (spgemm_set_allocator) or stream-ordered hipMallocAsync. Every
// buffer remembers the stream it was allocated on; it is freed on that stream
// after that stream has been made to wait for the plan's last work.
struct DevAllocator {
    spgemm_alloc_fn alloc = nullptr;
    spgemm_free_fn free = nullptr;
    void *ctx = nullptr;
};

struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    hipStream_t stream = nullptr;
};

struct spgemm_plan_s {
    int device = -1;
    DevAllocator allocator;
    // a plan of the allocation-free entry point carves every device buffer
    // from a fixed region (the static scratch array) instead
    bool use_arena = false;
    char *arena = nullptr;
    size_t arena_size = 0, arena_off = 0;
    hipEvent_t order_ev = nullptr;  // orders one stream after another (no timing)
    spgemm_dtype dt = SPGEMM_F64;
    bool batched = false;
    int nprob = 0;
    Tune tune{};
    uint32_t flags = 0;
    std::vector<Prob> probs;  // host copy of the problem table
    int ncols = 0, ntiles = 0, nblk = 0;
    bool symbolic_ok = false;

    // device workspace (one allocation, carved)
    DevBuf ws;
    Hdr *hdr = nullptr;
    int32_t *op = nullptr, *binw = nullptr, *gnnz = nullptr, *col0s = nullptr;
    int4 *binlist = nullptr;
    int2 *E = nullptr;
    long long total_nnzb = 0;
    long long *colprod = nullptr;
    // per-product arrays (own allocation: the product count is known only
    // after the classification): row and destination of every product, and
    // the later list's occurrence indices and ranks
    DevBuf prod;
    int32_t *prow = nullptr;
    uint32_t *dst = nullptr;
    int32_t *lk = nullptr, *lr = nullptr, *tilestart = nullptr;
    int nptiles = 0;
    long long prod_total = 0;  // products the product-space arrays are carved for
    bool spec_ready = false;   // a planned symbolic launch may be tried
    // staging of the later products for the numeric phase (sized by their count)
    DevBuf stage;
    int32_t *lo = nullptr, *lpid = nullptr, *lkc = nullptr;
    void *lv = nullptr;
    long long later_total = 0;  // products that are not the first of their entry
    long long *gcp = nullptr, *bsum = nullptr, *totals = nullptr;
    Prob *table = nullptr;
    int4 *tiles = nullptr;
    int32_t *th = nullptr, *tmax = nullptr;
    long long *ttot = nullptr;
    int nbsum = 0;

    // pinned host mirror of the header and totals (raw, then as published
    // pairs), mapped for the device
    void *pinned = nullptr, *pinned_dev = nullptr;
    size_t pinned_bytes = 0;
    uint32_t pub_seq = 0;
    Hdr hdr_host{};
    std::vector<long long> totals_host;

    // table currently on the device (batched numeric uploads when it changes)
    std::vector<Prob> table_dev_copy;
    hipEvent_t upload_done = nullptr;

    // side streams (default priority) on which the accumulator kinds run
    // concurrently with the caller's stream; fork/join through events
    static constexpr int kSide = 3;
    hipStream_t side[kSide] = {nullptr, nullptr, nullptr};
    hipEvent_t fork_ev = nullptr, join_ev[kSide] = {nullptr, nullptr, nullptr};

    // backward: row view of B
    DevBuf bt;
    bool bt_ready = false;
    int *bt_err = nullptr;

    bool wide_keys = false;  // some problem has 2^20 rows or more: 64-bit sort keys
    bool wide_esc = false;   // some problem has 2^24 - 1 rows or more: 64-bit ESC keys
    bool wide_acc = false;   // some problem has 2^21 - 1 rows or more: 64-bit keys of the
                             // direct-gather accumulators

    // Direct-gather accumulators (the default: no hash-accumulator or
    // lane-hash option): no per-product arrays; heavy columns expand into a
    // scratch of heavy_cap products with win_cap window counts
    bool direct = true;
    long long *hoff = nullptr;
    int32_t *wbase = nullptr;
    int32_t *wcnt = nullptr, *hrow = nullptr, *winmap = nullptr;
    void *hval = nullptr;
    uint32_t *hperm = nullptr;  // radix-sort indices (SPGEMM_RADIX_ESC)
    int rowbits = 0;            // bits of the largest row index over the problems
    int maxm = 0;               // largest row count over the problems
    // lane-per-column blocks (SPGEMM_LANE_BLOCKED): sort, blocks and value slabs
    DevBuf lbuf;
    LbArgs lb{};
    int lb_grid = 0;            // wavefronts of the block launch (one value slab each)
    long long heavy_cap = 0;
    int32_t win_cap = 0;
    // the column pointers of the last structure (single problem): a
    // one-call product may run its numeric phase at these positions first
    int32_t *saved_cp = nullptr;
    bool saved_ok = false;
    long long saved_total = 0;

    hipStream_t last_stream = nullptr;
};

namespace {

constexpr int32_t kVersion = 10000;  // 1.0.0

// ---------------------------------------------------------------- profiling
struct ProfRec {
    const char *name;
    hipEvent_t a, b;
};
struct Profiler {
    bool on = false;
    char only[32] = {0};  // record only this launch group when set
    std::vector<ProfRec> recs;
    size_t used = 0;
} g_prof;

// Several scopes may be open at once (one per stream): a scope keeps the
// index of its record, which stays valid when the record list grows.
struct ProfScope {
    long ri = -1;
    hipStream_t s;
    ProfScope(const char *name, hipStream_t st) : s(st) {
        if (!g_prof.on) return;
        if (g_prof.only[0] && std::strncmp(g_prof.only, name, sizeof(g_prof.only)) != 0) return;
        if (g_prof.used == g_prof.recs.size()) {
            ProfRec nr{name, nullptr, nullptr};
            // timing only: a device-scope release keeps the events light
            if (hipEventCreateWithFlags(&nr.a, hipEventReleaseToDevice) != hipSuccess ||
                hipEventCreateWithFlags(&nr.b, hipEventReleaseToDevice) != hipSuccess)
                return;
            g_prof.recs.push_back(nr);
        }
        ri = (long)g_prof.used++;
        g_prof.recs[ri].name = name;
        (void)hipEventRecord(g_prof.recs[ri].a, s);
    }
    ~ProfScope() {
        if (ri >= 0) (void)hipEventRecord(g_prof.recs[ri].b, s);
    }
    ProfScope(const ProfScope &) = delete;
    ProfScope &operator=(const ProfScope &) = delete;
};

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }
constexpr size_t kHdrBytes = (sizeof(Hdr) + 63) / 64 * 64;  // header, then the totals
// The host mirror: the raw header and totals (pin bytes, read back by copies)
// and then the same words as published pairs (word, sequence number).
unsigned long long *pub_pairs_host(spgemm_plan p) {
    return (unsigned long long *)((char *)p->pinned + p->pinned_bytes);
}

// Queues the publication of the header and totals, tagged with the next
// sequence number; later work queued on s runs on behind it.
hipError_t publish(spgemm_plan p, hipStream_t s) {
    const uint32_t seq = ++p->pub_seq;
    return launch_publish(p->hdr, (int)((kHdrBytes + 8 * (size_t)p->nprob) / 4),
                          (char *)p->pinned_dev + p->pinned_bytes, seq, s);
}

// Waits until every published pair carries the last sequence number and
// copies the words to the raw mirror. The stream is polled now and then, so a
// failed or finished stream ends the wait.
spgemm_status wait_published(spgemm_plan p, hipStream_t s) {
    const int nwords = (int)((kHdrBytes + 8 * (size_t)p->nprob) / 4);
    const unsigned long long *pairs = pub_pairs_host(p);
    uint32_t *raw = (uint32_t *)p->pinned;
    unsigned spin = 0;
    for (int i = 0; i < nwords; ++i) {
        for (;;) {
            const unsigned long long v = __atomic_load_n(&pairs[i], __ATOMIC_ACQUIRE);
            if ((uint32_t)(v >> 32) == p->pub_seq) {
                raw[i] = (uint32_t)v;
                break;
            }
            if ((++spin & 1023u) == 0) {
                const hipError_t q = hipStreamQuery(s);
                // all queued work has ended: the pairs are written by now
                if (q == hipSuccess) {
                    const unsigned long long w = __atomic_load_n(&pairs[i], __ATOMIC_ACQUIRE);
                    if ((uint32_t)(w >> 32) != p->pub_seq) return SPGEMM_ERR_HIP;
                    raw[i] = (uint32_t)w;
                    break;
                }
                if (q != hipErrorNotReady) return SPGEMM_ERR_HIP;
            }
        }
    }
    return SPGEMM_OK;
}

spgemm_status hip_status(hipError_t e) {
    if (e == hipSuccess) return SPGEMM_OK;
    if (e == hipErrorOutOfMemory) return SPGEMM_ERR_NO_MEMORY;
    return SPGEMM_ERR_HIP;
}

#define SPG_TRY(expr)                                  \
    do {                                               \
        hipError_t e_ = (expr);                        \
        if (e_ != hipSuccess) return hip_status(e_);   \
    } while (0)

std::mutex g_alloc_mu;
DevAllocator g_alloc;  // process-wide choice for plans created from now on

DevAllocator current_allocator() {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    return g_alloc;
}

// stream `later` waits for the work queued so far on `earlier` (no host wait)
hipError_t order_after(spgemm_plan p, hipStream_t later, hipStream_t earlier) {
    if (later == earlier) return hipSuccess;
    if (!p->order_ev) {
        hipError_t e = hipEventCreateWithFlags(&p->order_ev,
                                               hipEventDisableTiming | hipEventReleaseToDevice);
        if (e != hipSuccess) return e;
    }
    hipError_t e = hipEventRecord(p->order_ev, earlier);
    if (e != hipSuccess) return e;
    return hipStreamWaitEvent(later, p->order_ev, 0);
}

// Releases b (its last use is ordered before the end of stream `s`).
void dev_free(spgemm_plan p, DevBuf &b, hipStream_t s) {
    if (!b.ptr) return;
    if (p->use_arena) {  // carved from the fixed region: nothing to return
        b = DevBuf{};
        return;
    }
    (void)order_after(p, b.stream, s);
    if (p->allocator.free) p->allocator.free(b.ptr, b.bytes, b.stream, p->allocator.ctx);
    else (void)hipFreeAsync(b.ptr, b.stream);
    b = DevBuf{};
}

// Replaces b by `bytes` of device memory usable in stream order on `s`
// (contents undefined). The old buffer's last use is ordered before the end
// of `s`, so nothing waits on the host.
spgemm_status dev_alloc(spgemm_plan p, DevBuf &b, size_t bytes, hipStream_t s) {
    dev_free(p, b, s);
    void *ptr = nullptr;
    if (p->use_arena) {
        const size_t off = (p->arena_off + 255) / 256 * 256;
        if (off > p->arena_size || bytes > p->arena_size - off) return SPGEMM_ERR_SCRATCH;
        ptr = p->arena + off;
        p->arena_off = off + bytes;
    } else if (p->allocator.alloc) {
        ptr = p->allocator.alloc(bytes, s, p->allocator.ctx);
    } else if (hipMallocAsync(&ptr, bytes, s) != hipSuccess) {
        (void)hipGetLastError();
        ptr = nullptr;
    }
    if (!ptr) return SPGEMM_ERR_NO_MEMORY;
    b.ptr = ptr;
    b.bytes = bytes;
    b.stream = s;
    return SPGEMM_OK;
}

spgemm_status resolve_options(const spgemm_options *opt, Tune &t, uint32_t &flags) {
    int t_esc = 256, t_dense = 1, dense_rows = 0, cap = 0, t_split = 2048, t_block = 0;
    int t_lane = kLbMaxT, b_min = 16, b_max = 64;
    flags = 0;
    if (opt) {
        if (opt->t_esc) t_esc = opt->t_esc;
        if (opt->t_dense) t_dense = opt->t_dense;
        dense_rows = opt->dense_rows;
        cap = opt->hash_cap;
        if (opt->t_split) t_split = opt->t_split;
        if (opt->t_block) t_block = opt->t_block;
        if (opt->t_lane) t_lane = opt->t_lane;
        if (opt->b_min) b_min = opt->b_min;
        if (opt->b_max) b_max = opt->b_max;
        flags = opt->flags;
    }
    if (flags & SPGEMM_LANE_SPARS) flags |= SPGEMM_LANE_BLOCKED;
    if (t_lane < 1 || t_lane > kLbMaxT) return SPGEMM_ERR_INVALID;
    if (b_min < 1 || b_max < b_min || b_max > 64) return SPGEMM_ERR_INVALID;
    if (t_esc < 4 || t_esc > kEscMaxProducts) return SPGEMM_ERR_INVALID;
    if (t_dense < 1) return SPGEMM_ERR_INVALID;
    if (dense_rows < 0) return SPGEMM_ERR_INVALID;
    if (cap != 0 && (cap < 16 || cap > (1 << 20))) return SPGEMM_ERR_INVALID;
    if (t_split < -1) return SPGEMM_ERR_INVALID;
    if (t_block < -1) return SPGEMM_ERR_INVALID;
    int bins = 1;
    while ((4 << (bins - 1)) < t_esc) ++bins;  // t_esc rounded up to a power of two
    t.esc_bins = bins;
    t.t_dense = t_dense;
    t.dense_rows = dense_rows;
    t.hash_cap = cap;
    t.t_split = t_split < 0 ? 0x7fffffff : t_split;
    t.t_block = t_block < 0 ? 0 : (t_block == 0 ? 0x7fffffff : t_block);
    t.t_lane = t_lane;
    t.b_min = b_min;
    t.b_max = b_max;
    return SPGEMM_OK;
}

spgemm_status check_desc(const spgemm_csc *m, bool need_val) {
    if (!m) return SPGEMM_ERR_NULL;
    if (m->nrows < 0 || m->ncols < 0 || m->nnz < 0) return SPGEMM_ERR_SHAPE;
    if (!m->colptr) return SPGEMM_ERR_NULL;
    if (m->nnz > 0 && !m->rowidx) return SPGEMM_ERR_NULL;
    if (need_val && m->nnz > 0 && !m->val) return SPGEMM_ERR_NULL;
    return SPGEMM_OK;
}

// Host-side CSC check including repeated rows (SPGEMM_VALIDATE).
spgemm_status validate_host(const spgemm_csc *m) {
    std::vector<int32_t> cp((size_t)m->ncols + 1), ri((size_t)m->nnz);
    if (hipMemcpy(cp.data(), m->colptr, cp.size() * 4, hipMemcpyDeviceToHost) != hipSuccess)
        return SPGEMM_ERR_HIP;
    if (m->nnz && hipMemcpy(ri.data(), m->rowidx, ri.size() * 4, hipMemcpyDeviceToHost) != hipSuccess)
        return SPGEMM_ERR_HIP;
    if (cp[0] != 0 || cp[m->ncols] != m->nnz) return SPGEMM_ERR_CSC;
    std::vector<int32_t> stamp((size_t)std::max(m->nrows, 1), -1);
    for (int32_t j = 0; j < m->ncols; ++j) {
        if (cp[j + 1] < cp[j]) return SPGEMM_ERR_CSC;
        for (int32_t p = cp[j]; p < cp[j + 1]; ++p) {
            int32_t r = ri[p];
            if (r < 0 || r >= m->nrows || stamp[r] == j) return SPGEMM_ERR_CSC;
            stamp[r] = j;
        }
    }
    return SPGEMM_OK;
}

// carve the workspace for the plan's current sizes; grows the allocation
spgemm_status ensure_workspace(spgemm_plan p, hipStream_t s) {
    const size_t n = (size_t)std::max(p->ncols, 1);
    p->nblk = ceil_div(std::max(p->ncols, 1), kScanBlock);
    p->nbsum = p->nblk + 2;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes, 256);
        return o;
    };
    // the header and the per-problem totals are adjacent: one copy reads both
    const size_t o_hdr = take(kHdrBytes + 8 * (size_t)std::max(p->nprob, 1));
    const size_t o_op = take(4 * n), o_binw = take(4 * n), o_binlist = take(16 * n),
                 o_gnnz = take(4 * n);
    const size_t o_E = take(8 * (size_t)std::max(p->total_nnzb, 1ll));
    const size_t o_colprod = take(8 * (n + 1));
    const size_t o_gcp = take(8 * (n + 1));
    const size_t o_bsum = take(8 * (size_t)p->nbsum);
    const size_t o_tab = take(sizeof(Prob) * (size_t)std::max(p->nprob, 1));
    const size_t o_c0 = take(4 * ((size_t)p->nprob + 1));
    const size_t o_tiles = take(sizeof(int4) * (size_t)std::max(p->ntiles, 1));
    const size_t o_th = take(4 * (size_t)NBINS * std::max(p->ntiles, 1));
    const size_t o_ttot = take(8 * (size_t)std::max(p->ntiles, 1));
    const size_t o_tmax = take(4 * (size_t)std::max(p->ntiles, 1));
    const size_t o_hoff = take(8 * (n + 1)), o_wbase = take(4 * (n + 1));
    const size_t o_saved = take(4 * (n + 1));
    const size_t need = off;
    if (need > p->ws.bytes) {
        if (spgemm_status st = dev_alloc(p, p->ws, need, s)) return st;
        p->table_dev_copy.clear();
        p->saved_ok = false;
    }
    char *b = (char *)p->ws.ptr;
    p->hdr = (Hdr *)(b + o_hdr);
    p->op = (int32_t *)(b + o_op);
    p->binw = (int32_t *)(b + o_binw);
    p->binlist = (int4 *)(b + o_binlist);
    p->gnnz = (int32_t *)(b + o_gnnz);
    p->E = (int2 *)(b + o_E);
    p->colprod = (long long *)(b + o_colprod);
    p->gcp = (long long *)(b + o_gcp);
    p->bsum = (long long *)(b + o_bsum);
    p->totals = (long long *)(b + o_hdr + kHdrBytes);
    p->table = (Prob *)(b + o_tab);
    p->col0s = (int32_t *)(b + o_c0);
    p->tiles = (int4 *)(b + o_tiles);
    p->th = (int32_t *)(b + o_th);
    p->ttot = (long long *)(b + o_ttot);
    p->tmax = (int32_t *)(b + o_tmax);
    p->hoff = (long long *)(b + o_hoff);
    p->wbase = (int32_t *)(b + o_wbase);
    p->saved_cp = (int32_t *)(b + o_saved);

    const size_t pin = kHdrBytes + 8 * (size_t)std::max(p->nprob, 1);
    if (pin > p->pinned_bytes && !p->use_arena) {
        if (p->pinned) (void)hipHostFree(p->pinned);
        p->pinned = p->pinned_dev = nullptr;
        p->pinned_bytes = 0;
        // coherent: the device's stores reach host memory without a copy
        if (hipHostMalloc(&p->pinned, 3 * pin, hipHostMallocMapped | hipHostMallocCoherent) !=
            hipSuccess)
            return SPGEMM_ERR_NO_MEMORY;
        if (hipHostGetDevicePointer(&p->pinned_dev, p->pinned, 0) != hipSuccess) {
            (void)hipHostFree(p->pinned);
            p->pinned = p->pinned_dev = nullptr;
            return SPGEMM_ERR_HIP;
        }
        p->pinned_bytes = pin;
        std::memset(p->pinned, 0, 3 * pin);
        p->pub_seq = 0;  // no pair carries the next number
    }
    return SPGEMM_OK;
}

KArgs make_args(spgemm_plan p) {
    KArgs a{};
    a.single = p->probs.empty() ? Prob{} : p->probs[0];
    a.table = p->table;
    a.col0s = p->col0s;
    a.nprob = p->nprob;
    a.ncols = p->ncols;
    a.ntiles = p->ntiles;
    a.tiles = p->tiles;
    a.th = p->th;
    a.ttot = p->ttot;
    a.tmax = p->tmax;
    a.tune = p->tune;
    a.hdr = p->hdr;
    a.op = p->op;
    a.binw = p->binw;
    a.binlist = p->binlist;
    a.gnnz = p->gnnz;
    a.E = p->E;
    a.colprod = p->colprod;
    a.prow = p->prow;
    a.dst = p->dst;
    a.tilestart = p->tilestart;
    a.nptiles = p->nptiles;
    a.prod_cap = p->prod_total;
    a.lk = p->lk;
    a.lr = p->lr;
    a.gcp = p->gcp;
    a.later_n = p->later_total;
    a.out_cap = 0x7fffffffffffffffll;
    a.lkc = p->lkc;
    a.lo = p->lo;
    a.lpid = p->lpid;
    a.lv = p->lv;
    a.hoff = p->hoff;
    a.wbase = p->wbase;
    a.wcnt = p->wcnt;
    a.winmap = p->winmap;
    a.hrow = p->hrow;
    a.hval = p->hval;
    a.hperm = p->hperm;
    a.heavy_cap = p->heavy_cap;
    a.win_cap = p->win_cap;
    return a;
}

int esc_groups(const Hdr &h) {
    int g = 0;
    for (int i = 0; i < kEscBins; ++i) g += ceil_div(h.bin_count[BIN_ESC0 + i], 64 >> i);
    return g;
}

int device_cus() {
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            cus <= 0)
            cus = 256;
    }
    return cus;
}

// One launch per accumulator kind, each with one wavefront (sort-merge) or
// one workgroup (dense, hash) per work item; the grids come from the bin sizes
// on the host.
hipError_t ensure_side_streams(spgemm_plan p) {
    if (p->fork_ev) return hipSuccess;
    hipError_t e;
    // the fork and join events only order streams of this device: a
    // device-scope release is enough (no write-back for the host's view)
    const unsigned ef = hipEventDisableTiming | hipEventReleaseToDevice;
    for (int i = 0; i < spgemm_plan_s::kSide; ++i) {
        if ((e = hipStreamCreateWithFlags(&p->side[i], hipStreamNonBlocking))) return e;
        if ((e = hipEventCreateWithFlags(&p->join_ev[i], ef))) return e;
    }
    return hipEventCreateWithFlags(&p->fork_ev, ef);
}


// side stream i, or the caller's stream when every kind runs on it
hipStream_t side(spgemm_plan p, int i, hipStream_t s) {
    return (p->flags & SPGEMM_ONE_STREAM) ? s : p->side[i];
}

// the side streams in `used` (bit i: side stream i) wait for the caller's
// stream, and later the caller's stream for them
hipError_t fork(spgemm_plan p, hipStream_t s, unsigned used) {
    if ((p->flags & SPGEMM_ONE_STREAM) || !used) return hipSuccess;
    hipError_t e;
    if ((e = hipEventRecord(p->fork_ev, s))) return e;
    for (int i = 0; i < spgemm_plan_s::kSide; ++i)
        if ((used >> i) & 1u)
            if ((e = hipStreamWaitEvent(p->side[i], p->fork_ev, 0))) return e;
    return hipSuccess;
}

// The side streams join in a chain (each used side waits on the previous
// one's end), so the caller's stream waits on one event: one barrier on the
// stream that usually ends last instead of one per side stream.
hipError_t join(spgemm_plan p, hipStream_t s, unsigned used) {
    if ((p->flags & SPGEMM_ONE_STREAM) || !used) return hipSuccess;
    hipError_t e;
    int prev = -1;
    for (int i = 0; i < spgemm_plan_s::kSide; ++i) {
        if (!((used >> i) & 1u)) continue;
        if (prev >= 0 && (e = hipStreamWaitEvent(p->side[i], p->join_ev[prev], 0))) return e;
        if ((e = hipEventRecord(p->join_ev[i], p->side[i]))) return e;
        prev = i;
    }
    return hipStreamWaitEvent(s, p->join_ev[prev], 0);
}

// first bin-list position of bin b
int bin_start(const Hdr &h, int b) {
    int f = 0;
    for (int i = 0; i < b; ++i) f += h.bin_count[i];
    return f;
}

// Symbolic accumulators. The kinds work on disjoint columns and run
// concurrently so their latencies overlap: the windowed sort of the largest
// columns (few, long workgroups that need a whole compute unit's LDS share)
// starts first on the caller's stream, which needs no event wait, followed by
// the two smaller sorts; the wavefront sort-merge sub-bins (and the workgroup
// hash classes when enabled) take one side stream, the two larger sorts
// another.
hipError_t launch_symbolic_accumulators(spgemm_plan p, const KArgs &a, hipStream_t s) {
    const Hdr &h = p->hdr_host;
    hipError_t e;
    // stream of each ESC sub-bin and sort class (-1: the caller's, after the
    // ESC sub-bins; sorts on side streams start first, largest class first)
    static const int esc_side = 0;  // stream of the ESC launch (-1: the caller's)
    static const int sort_stream[kSortBins] = {-1, -1, 1, 1};
    static const int wsort_stream = -1;
    unsigned used = 0;
    for (int c = 0; c < kBlkBins; ++c)
        if (h.bin_count[BIN_BLK0 + c]) used |= c == kBlkBins - 1 ? 4u : 1u;
    if (h.bin_count[BIN_WSORT] && wsort_stream >= 0) used |= 1u << wsort_stream;
    for (int c = 0; c < kSortBins; ++c)
        if (h.bin_count[BIN_SORT0 + c] && sort_stream[c] >= 0) used |= 1u << sort_stream[c];
    for (int i = 0; i < kEscBins; ++i)
        if (h.bin_count[BIN_ESC0 + i] && esc_side >= 0) used |= 1u << esc_side;
    if ((e = fork(p, s, used))) return e;
    static const char *bnames[kBlkBins] = {"block512_symbolic", "block1k_symbolic",
                                           "block2k_symbolic", "block4k_symbolic",
                                           "block_xl_symbolic"};
    for (int c = kBlkBins - 1; c >= 0; --c) {
        const int n = h.bin_count[BIN_BLK0 + c];
        if (!n) continue;
        hipStream_t sc = side(p, c == kBlkBins - 1 ? 2 : 0, s);
        ProfScope ps(bnames[c], sc);
        if ((e = launch_block(a, c, n, sc))) return e;
    }
    if (const int n = h.bin_count[BIN_WSORT]) {
        hipStream_t sw = wsort_stream < 0 ? s : side(p, wsort_stream, s);
        ProfScope ps("wsort_symbolic", sw);
        if ((e = launch_wsort(a, p->wide_keys, n, sw))) return e;
    }
    static const char *snames[kSortBins] = {"sort512_symbolic", "sort1k_symbolic",
                                            "sort2k_symbolic", "sort4k_symbolic"};
    for (int c = kSortBins - 1; c >= 0; --c) {
        const int n = h.bin_count[BIN_SORT0 + c];
        if (!n || sort_stream[c] < 0) continue;
        hipStream_t sc = side(p, sort_stream[c], s);
        ProfScope ps(snames[c], sc);
        if ((e = launch_sort(a, c, p->wide_keys, n, sc))) return e;
    }
    const bool lane = (p->flags & SPGEMM_LANE_HASH) != 0;
    {
        // on one stream, one launch over the sub-bins saves six kernel
        // boundaries; beside the other kinds, one launch per sub-bin (largest
        // first) shares the chip better (measured both ways)
        int groups[kEscBins];
        for (int i = 0; i < kEscBins; ++i)
            groups[i] = (lane && i <= kLaneMaxSub) ? 0 : ceil_div(h.bin_count[BIN_ESC0 + i], 64 >> i);
        hipStream_t se = esc_side < 0 ? s : side(p, esc_side, s);
        ProfScope ps("esc_symbolic", se);
        if (p->flags & SPGEMM_ONE_STREAM) {
            if ((e = launch_esc_all(a, p->wide_esc, groups, se))) return e;
        } else {
            for (int i = kEscBins - 1; i >= 0; --i)
                if (groups[i] && (e = launch_esc(a, p->wide_esc, i, groups[i], se))) return e;
        }
    }
    if (lane) {
        ProfScope ps("lane_symbolic", s);
        for (int i = kLaneMaxSub; i >= 0; --i) {
            hipStream_t si = esc_side < 0 ? s : side(p, esc_side, s);
            if ((e = launch_lane(a, i, h.bin_count[BIN_ESC0 + i], si))) return e;
        }
    }
    for (int c = 0; c < kSortBins; ++c) {
        const int n = h.bin_count[BIN_SORT0 + c];
        if (!n || sort_stream[c] >= 0) continue;
        ProfScope ps(snames[c], s);
        if ((e = launch_sort(a, c, p->wide_keys, n, s))) return e;
    }
    return join(p, s, used);
}

// Scratch of the direct-gather accumulators' heavy columns: rows and values
// of `prod` products and the counts of `win` windows. The capacities only grow
// and the layout follows them (not this call's sizes): a launch planned from
// an earlier call may use all of them.
spgemm_status ensure_heavy(spgemm_plan p, long long prod, int win, hipStream_t s) {
    const size_t P = (size_t)std::max<long long>({prod, 1, p->heavy_cap});
    const size_t Wn = (size_t)std::max({win, 1, p->win_cap});
    const size_t o_val = align_up(4 * P, 256), o_win = o_val + align_up(8 * P, 256);
    const size_t o_map = o_win + align_up(4 * Wn, 256);
    // two index arrays of the radix sort (SPGEMM_RADIX_ESC)
    const size_t o_perm = o_map + align_up(4 * Wn, 256);
    const size_t need = (p->flags & SPGEMM_RADIX_ESC) ? o_perm + 8 * P : o_map + 4 * Wn;
    if (need > p->prod.bytes)
        if (spgemm_status st = dev_alloc(p, p->prod, need, s)) return st;
    p->heavy_cap = (long long)P;
    p->win_cap = (int)Wn;
    char *b = (char *)p->prod.ptr;
    p->hrow = (int32_t *)b;
    p->hval = b + o_val;
    p->wcnt = (int32_t *)(b + o_win);
    p->winmap = (int32_t *)(b + o_map);
    p->hperm = (p->flags & SPGEMM_RADIX_ESC) ? (uint32_t *)(b + o_perm) : nullptr;
    return SPGEMM_OK;
}

// Lane-per-column blocks (SPGEMM_LANE_BLOCKED): the sort, the block
// descriptors and one value slab per wavefront of the block launch (128 slots
// of 64 lanes for HASH, all rows of 64 lanes for SPARS), at most 1 GiB of
// slabs and 2048 wavefronts. The Op histogram starts at zero and every launch leaves it so.
spgemm_status ensure_lblock(spgemm_plan p, hipStream_t s) {
    if (!(p->flags & SPGEMM_LANE_BLOCKED)) return SPGEMM_OK;
    const bool spars = (p->flags & SPGEMM_LANE_SPARS) != 0;
    if (spars && p->maxm > kSparsMaxRows) return SPGEMM_ERR_INVALID;
    int nsub = 1;
    while ((4 << (nsub - 1)) < p->tune.t_lane) ++nsub;
    nsub = std::min(nsub, p->tune.esc_bins);
    const int mslab = spars ? std::max(p->maxm, 1) : 0;
    const size_t slab = (size_t)(spars ? mslab : 2 * kLbMaxT) * 64 * 8;
    // the allocation-free entry point carves from a fixed array: 32 MiB of slabs there
    const size_t budget = p->use_arena ? ((size_t)32 << 20) : ((size_t)1 << 30);
    const int grid = (int)std::max<size_t>(1, std::min<size_t>(2048, budget / slab));
    // hist and pos: kLbMaxT + 1 ints each (Op values 1..t)
    const size_t o_pos = align_up(4 * (size_t)(kLbMaxT + 1), 256);
    const size_t o_cnt = o_pos + align_up(4 * (size_t)(kLbMaxT + 1), 256);
    const size_t o_desc = o_cnt + 256;
    const size_t o_sorted = align_up(o_desc + 16 * (size_t)kLbMaxDesc, 256);
    const size_t o_dense = align_up(o_sorted + 16 * (size_t)std::max(p->ncols, 1), 256);
    const size_t need = o_dense + (size_t)grid * slab;
    if (need > p->lbuf.bytes) {
        if (spgemm_status st = dev_alloc(p, p->lbuf, need, s)) return st;
        SPG_TRY(hipMemsetAsync(p->lbuf.ptr, 0, 4 * (kLbMaxT + 1), s));
    }
    char *b = (char *)p->lbuf.ptr;
    LbArgs &lb = p->lb;
    lb.t = 4 << (nsub - 1);
    lb.b_min = p->tune.b_min;
    lb.b_max = p->tune.b_max;
    lb.nsub = nsub;
    lb.mslab = mslab;
    lb.hist = (int32_t *)b;
    lb.pos = (int32_t *)(b + o_pos);
    lb.counts = (int32_t *)(b + o_cnt);
    lb.desc = (int4 *)(b + o_desc);
    lb.sorted = (int4 *)(b + o_sorted);
    lb.ncap = std::max(p->ncols, 1);
    lb.dense = b + o_dense;
    p->lb_grid = grid;
    return SPGEMM_OK;
}

// The direct-gather accumulators of every bin, counting (fill = false) or
// filling C, on three streams: the wavefront groups and lane bins of the
// columns of at most 64 products on one side stream, the wavefront groups of
// up to 256 and the one-column waves (up to 1024 products) on another, the
// heavy columns (above 1024 products) on the caller's. The host takes
// several microseconds per launch, so the order of the launches matters:
// first the heavy columns' plan when plan_heavy asks for it (a single
// workgroup that then runs before the accumulators fill the chip) and every
// launch of the heavy chain but its last, then one launch per stream in turn
// (each stream's first kernel early).
struct LaunchQueue {
    const char *name;
    hipStream_t st;
    std::vector<std::function<hipError_t()>> l;
    size_t next = 0;
    std::optional<ProfScope> ps;
};

hipError_t launch_direct_accumulators(spgemm_plan p, const KArgs &a, hipStream_t s, bool fill,
                                      bool plan_heavy) {
    const Hdr &h = p->hdr_host;
    const bool f64 = p->dt == SPGEMM_F64;
    const bool wide = p->wide_acc;
    hipError_t e;
    // a small product runs on the caller's stream alone: the events of a
    // fork and join cost more than the overlap gains
    const bool one = (p->flags & SPGEMM_ONE_STREAM) || h.total_op < kSmallProducts;
    auto on = [&](int i) { return one ? s : side(p, i, s); };
    unsigned used = 0;
    if (!one) {
        for (int i = 0; i < kEscBins; ++i)
            if (h.bin_count[BIN_ESC0 + i]) used |= i < kEscSide0 ? 1u : 2u;
        for (int c = 0; c < 2; ++c)
            if (h.bin_count[BIN_SORT0 + c]) used |= 2u;
    }
    if ((e = fork(p, s, used))) return e;
    if (plan_heavy) {
        ProfScope ps("heavy_plan", s);
        if ((e = launch_heavy_plan(a, s))) return e;
    }
    LaunchQueue q[3] = {{fill ? "esc_numeric" : "esc_symbolic", on(0), {}},
                        {fill ? "heavy_numeric" : "heavy_symbolic", s, {}},
                        {fill ? "wave_numeric" : "wave_symbolic", on(1), {}}};
    // side stream 0: the lightest sub-bins as lane-per-column blocks (option),
    // then the wavefront sub-bins from the largest down
    const bool lbk = (p->flags & SPGEMM_LANE_BLOCKED) != 0;
    if (lbk) {
        int nl = 0;
        for (int i = 0; i < p->lb.nsub; ++i) nl += h.bin_count[BIN_ESC0 + i];
        const bool spars = (p->flags & SPGEMM_LANE_SPARS) != 0;
        const hipStream_t se = q[0].st;
        q[0].l.push_back([=, &a] { return launch_lane_blocked(a, p->lb, nl, p->lb_grid, spars, fill, f64, se); });
    }
    // (the sub-bins above 64 products go to side stream 1, below)
    for (int i = std::min(kEscBins, kEscSide0) - 1; i >= 0; --i) {
        if (lbk && i < p->lb.nsub) continue;
        const int n = h.bin_count[BIN_ESC0 + i];
        const hipStream_t se = q[0].st;
        if (n)
            q[0].l.push_back([=, &a] {
                return launch_acc_wave(a, BIN_ESC0 + i, wave_bin_items(BIN_ESC0 + i, n), wide, fill,
                                       f64, se);
            });
    }
    // caller's stream: columns above 1024 products (bins SORT2, SORT3, WSORT)
    const int nheavy =
        h.bin_count[BIN_SORT2] + h.bin_count[BIN_SORT3] + h.bin_count[BIN_WSORT];
    if (nheavy) {
        const bool radix = (p->flags & SPGEMM_RADIX_ESC) != 0;
        const int nwin = h.heavy_win, rowbits = p->rowbits;
        const long long hp = (long long)h.heavy_prod;
        for (int part = heavy_first_part(radix, plan_heavy && a.spec_total >= 0);
             part < heavy_parts(radix); ++part)
            q[1].l.push_back([=, &a] {
                return launch_heavy(a, nheavy, nwin, wide, fill, f64, s, radix, hp, rowbits, part);
            });
    }
    // side stream 1: the one-column waves, 1024 products then 512, then the
    // wavefront sub-bins above 64 products (the three streams then hold
    // similar work on power-law inputs)
    for (int c = 1; c >= 0; --c) {
        const int n = h.bin_count[BIN_SORT0 + c];
        const hipStream_t sw = q[2].st;
        if (n) q[2].l.push_back([=, &a] { return launch_acc_wave(a, BIN_SORT0 + c, n, wide, fill, f64, sw); });
    }
    for (int i = kEscBins - 1; i >= kEscSide0; --i) {
        const int n = h.bin_count[BIN_ESC0 + i];
        const hipStream_t sw = q[2].st;
        if (n)
            q[2].l.push_back([=, &a] {
                return launch_acc_wave(a, BIN_ESC0 + i, wave_bin_items(BIN_ESC0 + i, n), wide, fill,
                                       f64, sw);
            });
    }
    // on one stream the queues go one after the other (nothing to overlap;
    // each launch group's timing events then bracket only its own kernels)
    const bool interleave = !one;
    // the heavy columns' chain is the longest: all its launches but the last
    // go before the side streams' first ones
    if (interleave) {
        LaunchQueue &x = q[1];
        while (x.next + 1 < x.l.size()) {
            if (x.next == 0) x.ps.emplace(x.name, x.st);
            if ((e = x.l[x.next++]())) return e;
        }
    }
    for (bool more = true; more;) {
        more = false;
        for (LaunchQueue &x : q) {
            while (x.next < x.l.size()) {
                if (x.next == 0) x.ps.emplace(x.name, x.st);
                if ((e = x.l[x.next++]())) return e;
                if (x.next == x.l.size()) x.ps.reset();
                more = true;
                if (interleave) break;
            }
        }
    }
    return join(p, s, used);
}

// Numeric: one launch over the tiles and the chunks of the columns above
// t_split, then one small launch per occurrence index of the later products.
// The sizes a numeric launch is planned from (the plan's header and later
// count): a numeric phase queued before they are read back is valid when
// they come back unchanged.
struct NumLaunch {
    int first = 0, nbig = 0, big_chunks = 0, later_maxk = 0, nptiles = 0;
    long long later_total = 0;
    bool operator==(const NumLaunch &o) const {
        return first == o.first && nbig == o.nbig && big_chunks == o.big_chunks &&
               later_maxk == o.later_maxk && nptiles == o.nptiles && later_total == o.later_total;
    }
};

NumLaunch numeric_launch(spgemm_plan p) {
    const Hdr &h = p->hdr_host;
    // columns above t_split: the bins from the first one whose largest
    // product count exceeds t_split on (bin-list order)
    int fb = BIN_ESC0;
    while (fb < NBINS) {
        const long long bmax = fb < BIN_SORT0   ? (4ll << (fb - BIN_ESC0))
                               : fb < BIN_WSORT ? (512ll << (fb - BIN_SORT0))
                               : fb == BIN_WSORT ? 0x7fffffffll
                               : fb < BIN_BLK4  ? (512ll << (fb - BIN_BLK0))
                                                : 0x7fffffffll;
        if (bmax > p->tune.t_split) break;
        ++fb;
    }
    NumLaunch L;
    L.first = bin_start(h, fb);
    for (int b = fb; b < NBINS; ++b) L.nbig += h.bin_count[b];
    L.big_chunks = h.big_chunks;
    L.later_maxk = h.later_maxk;
    L.later_total = p->later_total;
    L.nptiles = p->nptiles;
    return L;
}

hipError_t launch_numeric_phase(spgemm_plan p, const KArgs &a, hipStream_t s) {
    if (p->direct) return launch_direct_accumulators(p, a, s, true, false);
    const bool f64 = p->dt == SPGEMM_F64;
    const NumLaunch L = numeric_launch(p);
    hipError_t e;
    {
        ProfScope ps("numeric", s);
        if ((e = launch_numeric(a, f64, L.first, L.nbig, L.big_chunks, s))) return e;
    }
    if (L.later_total == 0) return hipSuccess;
    ProfScope ps("later_layers", s);
    // the hash accumulator numbers its later products in settling order; the
    // others in sorted-key order, where one launch adds them all
    bool hashed = false;
    for (int c = 0; c < kBlkBins; ++c) hashed |= p->hdr_host.bin_count[BIN_BLK0 + c] > 0;
    if (!hashed) return launch_later_runs(a, f64, L.later_total, s);
    for (int k = 1; k <= L.later_maxk; ++k)
        if ((e = launch_layer(a, f64, k, L.later_total, s))) return e;
    return hipSuccess;
}

// Product-space arrays for `total` products (the allocation only grows).
spgemm_status ensure_products(spgemm_plan p, unsigned long long total, hipStream_t s) {
    const size_t P = (size_t)std::max<unsigned long long>(total, 1);
    const size_t q1 = align_up(4 * P, 256);
    p->nptiles = (int)(total / kProdTile) + 1;
    const size_t pneed = 4 * q1 + 4 * ((size_t)p->nptiles + 1);
    if (pneed > p->prod.bytes)
        if (spgemm_status st = dev_alloc(p, p->prod, pneed, s)) return st;
    char *base = (char *)p->prod.ptr;
    p->prow = (int32_t *)base;
    p->dst = (uint32_t *)(base + q1);
    p->lk = (int32_t *)(base + 2 * q1);
    p->lr = (int32_t *)(base + 3 * q1);
    p->tilestart = (int32_t *)(base + 4 * q1);
    p->prod_total = (long long)total;
    return SPGEMM_OK;
}

// One pass of the symbolic launch sequence; returns after the totals are on
// the host. A planned pass (spec) launches everything from the sizes of the
// plan's previous call with no read-back in between; when the device finds
// other sizes it does no product-space work and *retry is set.
// Outputs of a one-call product (spgemm_multiply): in a planned pass the
// numeric phase is queued right behind the symbolic one, from the previous
// call's sizes, and the host waits only for the header read-back.
struct FusedOut {
    int32_t *cri;
    void *cv;
    long long cap;
    bool queued;   // a numeric phase was queued in this call's planned pass
    NumLaunch used;
};

spgemm_status symbolic_pass(spgemm_plan p, hipStream_t s, const std::vector<int4> &tiles_host,
                            bool spec, bool *retry, FusedOut *fo) {
    *retry = false;
    spgemm_status st = ensure_workspace(p, s);
    if (st) return st;
    if (p->nprob > 1) {
        std::vector<int32_t> c0(p->nprob + 1);
        for (int i = 0; i < p->nprob; ++i) c0[i] = p->probs[i].col0;
        c0[p->nprob] = p->ncols;
        SPG_TRY(hipMemcpyAsync(p->table, p->probs.data(), sizeof(Prob) * p->nprob,
                               hipMemcpyHostToDevice, s));
        SPG_TRY(hipMemcpyAsync(p->col0s, c0.data(), 4 * c0.size(), hipMemcpyHostToDevice, s));
        SPG_TRY(hipMemcpyAsync(p->tiles, tiles_host.data(), sizeof(int4) * tiles_host.size(),
                               hipMemcpyHostToDevice, s));
        // the pageable sources may change after return: wait for the copies
        SPG_TRY(hipStreamSynchronize(s));
        p->table_dev_copy = p->probs;
    }
    SPG_TRY(hipMemsetAsync(p->hdr, 0, sizeof(Hdr), s));
    // launches are planned from hdr_host: the previous call's sizes (spec) or
    // this call's, read back after the placement
    unsigned mask = 0;
    for (int b = 0; b < NBINS; ++b) mask |= (p->hdr_host.bin_count[b] > 0 ? 1u : 0u) << b;
    auto args = [&]() {
        KArgs a = make_args(p);
        a.spec_total = spec ? p->prod_total : -1;
        a.spec_mask = spec ? mask : 0u;
        if (spec && fo) a.out_cap = fo->cap;
        return a;
    };
    // A planned launch runs the tally and the placement (needed only by the
    // accumulators) on a side stream while the product offsets and the
    // expansion run on the caller's; the offsets kernel stops the expansion if
    // the products outgrow the planned product space.
    // (The direct-gather accumulators have nothing to overlap them with.)
    const bool overlap = spec && !p->direct && p->ncols > 0 && !(p->flags & SPGEMM_ONE_STREAM);
    {
        const KArgs a = args();
        { ProfScope ps("classify", s); SPG_TRY(launch_classify(a, s)); }
        if (overlap) SPG_TRY(fork(p, s, 1u));
        hipStream_t sp = overlap ? p->side[0] : s;
        { ProfScope ps("tally", sp); SPG_TRY(launch_tally(a, sp)); }
        { ProfScope ps("place", sp); SPG_TRY(launch_place(a, sp)); }
        // a planned launch queues the heavy columns' plan behind the fork of
        // the accumulator streams; a first launch reads its totals back here
        if (p->direct && p->ncols > 0 && !spec) {
            ProfScope ps("heavy_plan", s);
            SPG_TRY(launch_heavy_plan(a, s));
        }
    }
    if (!spec) {
        // the bin sizes fix the grids and the product count the allocation
        SPG_TRY(hipMemcpyAsync(p->pinned, p->hdr, sizeof(Hdr), hipMemcpyDeviceToHost, s));
        SPG_TRY(hipStreamSynchronize(s));
        std::memcpy(&p->hdr_host, p->pinned, sizeof(Hdr));
        const int err = p->hdr_host.err;
        if (err & ERR_CSC) return SPGEMM_ERR_CSC;
        if (err & ERR_OPOVF) return SPGEMM_ERR_INDEX_OVERFLOW;
        if (p->direct) {
            if ((st = ensure_heavy(p, (long long)p->hdr_host.heavy_prod, p->hdr_host.heavy_win, s)))
                return st;
        } else if ((st = ensure_products(p, p->hdr_host.total_op, s))) {
            return st;
        }
    }
    // A planned one-call product on a plan whose last structure is known runs
    // its numeric phase now, at that structure's column positions, counting
    // every column's entries as it goes; the scan then builds this call's
    // column pointers from those counts. A count that differs asks for a redo.
    const bool speculate = p->direct && spec && fo && p->nprob == 1 && p->saved_ok &&
                           p->saved_total <= fo->cap && p->ncols > 0;
    if (p->ncols > 0 && p->direct) {
        if ((st = ensure_lblock(p, s))) return st;
        const KArgs al = args();
        if (speculate) {
            KArgs af = al;
            af.single.cri = fo->cri;
            af.single.cv = fo->cv;
            af.single.ccp = p->saved_cp;
            af.spec_fill = 1;
            SPG_TRY(launch_direct_accumulators(p, af, s, true, true));
            fo->queued = true;
            fo->used = numeric_launch(p);
        } else {
            SPG_TRY(launch_direct_accumulators(p, al, s, false, spec));
        }
        ProfScope ps("scan", s);
        SPG_TRY(launch_scan(al, p->gcp, p->bsum, p->nblk, p->totals, s));
    } else if (p->ncols > 0) {
        const KArgs al = args();
        {
            // first product of every column (exclusive scan of Op_j), tiles
            ProfScope ps("product_offsets", s);
            SPG_TRY(launch_prod_offsets(al, p->bsum, p->nbsum, s));
        }
        { ProfScope ps("expand", s); SPG_TRY(launch_expand(al, s)); }
        if (overlap) SPG_TRY(join(p, s, 1u));
        SPG_TRY(launch_symbolic_accumulators(p, al, s));
        ProfScope ps("scan", s);
        SPG_TRY(launch_scan(al, p->gcp, p->bsum, p->nblk, p->totals, s));
    }
    if (p->use_arena) {
        // no mapped host memory: a plain copy of the header and totals to the
        // plan's host buffer, then a wait
        SPG_TRY(hipMemcpyAsync(p->pinned, p->hdr, kHdrBytes + 8 * (size_t)p->nprob,
                               hipMemcpyDeviceToHost, s));
        SPG_TRY(hipStreamSynchronize(s));
    } else {
        SPG_TRY(publish(p, s));
    }
    if (fo && spec && p->ncols > 0 && p->nprob == 1 && !speculate) {
        // the numeric phase from the previous sizes; it stands down on an
        // error or capacity flag raised above, and is redone by the caller if
        // the sizes read back differ
        p->probs[0].cri = fo->cri;
        p->probs[0].cv = fo->cv;
        KArgs an = make_args(p);
        an.out_cap = fo->cap;
        fo->used = numeric_launch(p);
        fo->queued = true;
        SPG_TRY(launch_numeric_phase(p, an, s));
    }
    if (!p->use_arena) {
        const spgemm_status w = wait_published(p, s);
        if (w != SPGEMM_OK) return w;
    }
    std::memcpy(&p->hdr_host, p->pinned, sizeof(Hdr));
    int err = p->hdr_host.err;
    if (err & ERR_CSC) return SPGEMM_ERR_CSC;
    if (err & ERR_OPOVF) return SPGEMM_ERR_INDEX_OVERFLOW;
    if (spec && (err & ERR_RETRY)) {
        *retry = true;
        return SPGEMM_OK;
    }
    p->totals_host.assign(p->nprob, 0);
    if (p->ncols > 0)
        std::memcpy(p->totals_host.data(), (char *)p->pinned + kHdrBytes, 8 * (size_t)p->nprob);
    if (err & (ERR_GROUP | ERR_RETRY)) return SPGEMM_ERR_CSC;
    if (err & ERR_NNZOVF) return SPGEMM_ERR_INDEX_OVERFLOW;
    // products beyond the first of their entry (the staged later products of
    // the product-space accumulators)
    long long nnz_all = 0;
    for (long long t : p->totals_host) nnz_all += t;
    p->later_total = (long long)p->hdr_host.total_op - nnz_all;
    if (p->later_total < 0) return SPGEMM_ERR_CSC;  // cannot happen
    if (p->direct) {
        // a later planned pass compares its product total with this one
        p->prod_total = (long long)p->hdr_host.total_op;
        if (p->nprob == 1 && p->ncols > 0 && !speculate) {
            // the structure a later one-call product may start from
            SPG_TRY(hipMemcpyAsync(p->saved_cp, p->probs[0].ccp, 4 * ((size_t)p->ncols + 1),
                                   hipMemcpyDeviceToDevice, s));
            p->saved_total = p->totals_host[0];
            p->saved_ok = true;
        }
        if (p->ncols == 0) {
            for (int i = 0; i < p->nprob; ++i)
                SPG_TRY(hipMemsetAsync(p->probs[i].ccp, 0, sizeof(int32_t), s));
            SPG_TRY(hipStreamSynchronize(s));
        }
        p->symbolic_ok = true;
        p->spec_ready = p->ncols > 0;
        return SPGEMM_OK;
    }
    const size_t NL = (size_t)std::max<long long>(p->later_total, 1);
    const size_t vsz = p->dt == SPGEMM_F64 ? 8 : 4;
    const size_t o_pid = align_up(4 * NL, 256), o_k = o_pid + align_up(4 * NL, 256);
    const size_t o_v = o_k + align_up(4 * NL, 256);
    const size_t sneed = o_v + vsz * NL;
    if (sneed > p->stage.bytes) {
        // a numeric phase queued behind this pass still reads the old
        // staging: it is released in stream order behind it
        if ((st = dev_alloc(p, p->stage, sneed, s))) return st;
    }
    char *sb = (char *)p->stage.ptr;
    p->lo = (int32_t *)sb;
    p->lpid = (int32_t *)(sb + o_pid);
    p->lkc = (int32_t *)(sb + o_k);
    p->lv = sb + o_v;
    if (p->ncols == 0) {
        // no columns at all: every problem's column pointer is {0}
        for (int i = 0; i < p->nprob; ++i)
            SPG_TRY(hipMemsetAsync(p->probs[i].ccp, 0, sizeof(int32_t), s));
        SPG_TRY(hipStreamSynchronize(s));
    }
    p->symbolic_ok = true;
    p->spec_ready = p->ncols > 0;
    return SPGEMM_OK;
}

// Symbolic phase: a planned pass when the plan has run before, the pass with
// the mid read-back when it has not or when the sizes changed.
spgemm_status run_symbolic(spgemm_plan p, hipStream_t s, const std::vector<int4> &tiles_host,
                           FusedOut *fo) {
    bool retry = false;
    if (p->spec_ready && !(p->flags & SPGEMM_NO_PLANNED_LAUNCH)) {
        const spgemm_status st = symbolic_pass(p, s, tiles_host, true, &retry, fo);
        if (st || !retry) {
            if (st) p->spec_ready = false;
            return st;
        }
    }
    p->spec_ready = false;
    if (fo && fo->queued) {
        // the queued numeric phase stood down; let it drain before the redo
        // may reallocate what it reads
        SPG_TRY(hipStreamSynchronize(s));
        fo->queued = false;
    }
    return symbolic_pass(p, s, tiles_host, false, &retry, fo);
}

spgemm_status run_numeric(spgemm_plan p, hipStream_t s) {
    const KArgs a = make_args(p);
    SPG_TRY(launch_numeric_phase(p, a, s));
    p->last_stream = s;
    return SPGEMM_OK;
}

spgemm_plan get_or_new_plan(spgemm_plan *inout) {
    if (*inout) return *inout;
    return new (std::nothrow) spgemm_plan_s();
}

}  // namespace

extern "C" {

const char *spgemm_status_string(spgemm_status s) {
    switch (s) {
        case SPGEMM_OK: return "ok";
        case SPGEMM_ERR_NULL: return "null pointer";
        case SPGEMM_ERR_SHAPE: return "shape mismatch";
        case SPGEMM_ERR_CSC: return "malformed CSC input";
        case SPGEMM_ERR_DTYPE: return "unknown value type";
        case SPGEMM_ERR_INDEX_OVERFLOW: return "index overflow (int32)";
        case SPGEMM_ERR_NO_MEMORY: return "out of memory";
        case SPGEMM_ERR_HIP: return "HIP runtime error";
        case SPGEMM_ERR_PLAN: return "invalid plan";
        case SPGEMM_ERR_INVALID: return "invalid argument";
        case SPGEMM_ERR_NOT_TUNED: return "no tuning cache entry for the workload";
        case SPGEMM_ERR_CAPACITY: return "C arrays smaller than nnz(C)";
        case SPGEMM_ERR_SCRATCH:
            return "problem needs more workspace than the static scratch array holds";
    }
    return "unknown status";
}

int32_t spgemm_version(void) { return kVersion; }

static spgemm_status symbolic_common(int32_t count, const spgemm_csc *A, const spgemm_csc *B,
                                     spgemm_dtype dt, const spgemm_options *opt, void *stream,
                                     spgemm_plan *plan_inout, int32_t *const *C_colptr,
                                     int64_t *nnzC_host, bool batched, FusedOut *fo = nullptr) {
    if (!plan_inout || !A || !B || !C_colptr || !nnzC_host) return SPGEMM_ERR_NULL;
    if (dt != SPGEMM_F32 && dt != SPGEMM_F64) return SPGEMM_ERR_DTYPE;
    if (count < 0) return SPGEMM_ERR_INVALID;
    Tune tune;
    uint32_t flags;
    spgemm_status st = resolve_options(opt, tune, flags);
    if (st) return st;
    long long ncols = 0, nnzb_total = 0;
    std::vector<Prob> probs(count);
    std::vector<int4> tiles;
    for (int i = 0; i < count; ++i) {
        if ((st = check_desc(&A[i], false)) || (st = check_desc(&B[i], false))) return st;
        if (!C_colptr[i]) return SPGEMM_ERR_NULL;
        if (A[i].ncols != B[i].nrows) return SPGEMM_ERR_SHAPE;
        if (flags & SPGEMM_VALIDATE) {
            if ((st = validate_host(&A[i])) || (st = validate_host(&B[i]))) return st;
        }
        Prob &q = probs[i];
        q = Prob{};
        q.m = A[i].nrows; q.k = A[i].ncols; q.n = B[i].ncols;
        q.col0 = (int32_t)ncols;
        q.nnza = A[i].nnz; q.nnzb = B[i].nnz;
        q.ebase = nnzb_total;
        nnzb_total += q.nnzb;
        q.acp = A[i].colptr; q.ari = A[i].rowidx; q.av = A[i].val;
        q.bcp = B[i].colptr; q.bri = B[i].rowidx; q.bv = B[i].val;
        q.ccp = C_colptr[i];
        for (int j0 = 0; j0 < q.n; j0 += kTile)
            tiles.push_back(make_int4(i, j0, std::min(q.n, j0 + kTile), 0));
        ncols += q.n;
        if (ncols > 0x7fffffffll) return SPGEMM_ERR_INDEX_OVERFLOW;
    }
    spgemm_plan p = get_or_new_plan(plan_inout);
    if (!p) return SPGEMM_ERR_NO_MEMORY;
    const bool fresh = (*plan_inout == nullptr);
    if (fresh) p->allocator = current_allocator();
    p->dt = dt;
    p->batched = batched;
    p->nprob = count;
    p->tune = tune;
    p->flags = flags;
    p->probs = std::move(probs);
    // 32-bit sort keys (row << 12 | position) hold rows below 2^20 - 1: at
    // m = 2^20 the key of row 2^20 - 1 at position 4095 would equal the
    // all-ones padding key
    p->wide_keys = false;
    p->wide_esc = false;
    p->wide_acc = false;
    p->rowbits = 0;
    p->maxm = 0;
    for (const Prob &q : p->probs) {
        p->maxm = std::max(p->maxm, q.m);
        p->wide_keys |= q.m >= (1 << 20);
        p->wide_esc |= q.m >= (1 << 24) - 1;
        p->wide_acc |= q.m >= (1 << 21) - 1;
        p->rowbits = std::max(p->rowbits, row_bits(q.m));
    }
    // the hash accumulator and the lane-per-column hash run on the product
    // space; every other choice on the direct-gather accumulators
    const bool direct = tune.t_block == 0x7fffffff && !(flags & SPGEMM_LANE_HASH);
    if (!fresh && direct != p->direct) p->spec_ready = false;
    p->direct = direct;
    p->ncols = (int)ncols;
    p->total_nnzb = nnzb_total;
    p->ntiles = (int)tiles.size();
    p->symbolic_ok = false;
    p->bt_ready = false;
    (void)hipGetDevice(&p->device);
    hipStream_t s = (hipStream_t)stream;
    if (count == 0) {
        *plan_inout = p;
        p->symbolic_ok = true;
        p->hdr_host = Hdr{};
        return SPGEMM_OK;
    }
    if (hipError_t e = ensure_side_streams(p)) {
        if (fresh) spgemm_plan_destroy(p);
        return hip_status(e);
    }
    // the plan's earlier work (possibly on another stream) comes first
    if (!fresh && p->last_stream != s)
        if (hipError_t e = order_after(p, s, p->last_stream)) return hip_status(e);
    st = run_symbolic(p, s, tiles, fo);
    p->last_stream = s;
    if (st) {
        if (fresh) spgemm_plan_destroy(p);
        else p->symbolic_ok = false;
        return st;
    }
    for (int i = 0; i < count; ++i) nnzC_host[i] = p->totals_host[i];
    *plan_inout = p;
    return SPGEMM_OK;
}

spgemm_status spgemm_symbolic(const spgemm_csc *A, const spgemm_csc *B, spgemm_dtype dt,
                              const spgemm_options *opt, void *stream, spgemm_plan *plan_inout,
                              int32_t *C_colptr, int64_t *nnzC_host) {
    if (!C_colptr) return SPGEMM_ERR_NULL;
    int32_t *cps[1] = {C_colptr};
    return symbolic_common(1, A, B, dt, opt, stream, plan_inout, cps, nnzC_host, false);
}

spgemm_status spgemm_numeric(spgemm_plan p, const void *A_val, const void *B_val,
                             int32_t *C_rowidx, void *C_val, void *stream) {
    if (!p) return SPGEMM_ERR_PLAN;
    if (p->batched || p->nprob != 1 || !p->symbolic_ok) return SPGEMM_ERR_PLAN;
    Prob &q = p->probs[0];
    const long long nnzc = p->totals_host[0];
    if ((q.nnza > 0 && !A_val) || (q.nnzb > 0 && !B_val)) return SPGEMM_ERR_NULL;
    if (nnzc > 0 && (!C_rowidx || !C_val)) return SPGEMM_ERR_NULL;
    q.av = A_val;
    q.bv = B_val;
    q.cri = C_rowidx;
    q.cv = C_val;
    if (nnzc == 0) return SPGEMM_OK;
    return run_numeric(p, (hipStream_t)stream);
}

spgemm_status spgemm_multiply(const spgemm_csc *A, const spgemm_csc *B, spgemm_dtype dt,
                              const spgemm_options *opt, void *stream, spgemm_plan *plan_inout,
                              int32_t *C_colptr, int32_t *C_rowidx, void *C_val, int64_t capacity,
                              int64_t *nnzC_host) {
    if (!A || !B || !C_colptr || !nnzC_host || !plan_inout) return SPGEMM_ERR_NULL;
    if (capacity < 0) return SPGEMM_ERR_INVALID;
    if ((A->nnz > 0 && !A->val) || (B->nnz > 0 && !B->val)) return SPGEMM_ERR_NULL;
    if (capacity > 0 && (!C_rowidx || !C_val)) return SPGEMM_ERR_NULL;
    hipStream_t s = (hipStream_t)stream;
    FusedOut fo{C_rowidx, C_val, (long long)capacity, false, NumLaunch{}};
    int32_t *cps[1] = {C_colptr};
    spgemm_status st = symbolic_common(1, A, B, dt, opt, stream, plan_inout, cps, nnzC_host, false,
                                       &fo);
    if (st) return st;
    spgemm_plan p = *plan_inout;
    const long long nnzc = p->totals_host.empty() ? 0 : p->totals_host[0];
    if (nnzc > capacity) {
        // the queued numeric phase stood down; clear its flag for later calls
        if (fo.queued) SPG_TRY(hipMemsetAsync(&p->hdr->cap_over, 0, sizeof(int32_t), s));
        return SPGEMM_ERR_CAPACITY;
    }
    Prob &q = p->probs[0];
    q.av = A->val;
    q.bv = B->val;
    q.cri = C_rowidx;
    q.cv = C_val;
    if (nnzc == 0) return SPGEMM_OK;
    if (fo.queued) {
        // already queued and valid: the direct-gather accumulators cover any
        // sizes from any grid; the others were planned from the same sizes
        if (p->direct || fo.used == numeric_launch(p)) return SPGEMM_OK;
        // queued from other sizes: its bounds checks may have raised the group
        // flag, which would make the phase below stand down; clear it first
        SPG_TRY(hipMemsetAsync(&p->hdr->err, 0, sizeof(int32_t), s));
    }
    return run_numeric(p, s);
}

spgemm_status spgemm_batched(int32_t count, const spgemm_csc *A_host, const spgemm_csc *B_host,
                             spgemm_dtype dt, const spgemm_options *opt, void *stream,
                             spgemm_plan *plan_inout, int32_t *const *C_colptr_host,
                             int64_t *nnzC_host, int32_t *const *C_rowidx_host,
                             void *const *C_val_host) {
    if (!plan_inout) return SPGEMM_ERR_NULL;
    if (!C_rowidx_host) {
        if (count == 1) {
            // one problem still runs through the batched (table) path
        }
        return symbolic_common(count, A_host, B_host, dt, opt, stream, plan_inout, C_colptr_host,
                               nnzC_host, true);
    }
    spgemm_plan p = *plan_inout;
    if (!p || !p->batched || !p->symbolic_ok || p->nprob != count || p->dt != dt)
        return SPGEMM_ERR_PLAN;
    if (!A_host || !B_host || !C_val_host) return SPGEMM_ERR_NULL;
    hipStream_t s = (hipStream_t)stream;
    for (int i = 0; i < count; ++i) {
        Prob &q = p->probs[i];
        if (A_host[i].nnz != q.nnza || B_host[i].nnz != q.nnzb) return SPGEMM_ERR_PLAN;
        if ((q.nnza > 0 && !A_host[i].val) || (q.nnzb > 0 && !B_host[i].val)) return SPGEMM_ERR_NULL;
        if (p->totals_host[i] > 0 && (!C_rowidx_host[i] || !C_val_host[i])) return SPGEMM_ERR_NULL;
        q.av = A_host[i].val;
        q.bv = B_host[i].val;
        q.cri = C_rowidx_host[i];
        q.cv = C_val_host[i];
    }
    if (count == 0) return SPGEMM_OK;
    if (count > 1) {
        bool same = p->table_dev_copy.size() == p->probs.size() &&
                    std::memcmp(p->table_dev_copy.data(), p->probs.data(),
                                sizeof(Prob) * p->probs.size()) == 0;
        if (!same) {
            SPG_TRY(hipMemcpyAsync(p->table, p->probs.data(), sizeof(Prob) * p->nprob,
                                   hipMemcpyHostToDevice, s));
            // the pageable source may be reused by the caller: wait for the copy
            SPG_TRY(hipStreamSynchronize(s));
            p->table_dev_copy = p->probs;
        }
    }
    return run_numeric(p, s);
}

spgemm_status spgemm_backward(spgemm_plan p, const void *A_val, const void *B_val,
                              const int32_t *C_rowidx, const void *G_val, void *dA_val,
                              void *dB_val, void *stream) {
    if (!p) return SPGEMM_ERR_PLAN;
    if (p->nprob != 1 || !p->symbolic_ok) return SPGEMM_ERR_PLAN;
    const Prob &q0 = p->probs[0];
    if (!dA_val && !dB_val) return SPGEMM_OK;
    if ((q0.nnza > 0 && !A_val && dB_val) || (q0.nnzb > 0 && !B_val && dA_val)) return SPGEMM_ERR_NULL;
    if (p->totals_host[0] > 0 && (!C_rowidx || !G_val)) return SPGEMM_ERR_NULL;
    hipStream_t s = (hipStream_t)stream;
    Prob q = q0;
    q.av = A_val;
    q.bv = B_val;
    const bool f64 = p->dt == SPGEMM_F64;
    // the backward view (per B entry, per A entry, row view of B), its
    // construction temporaries, scan partials and an error word
    const size_t k = (size_t)q.k, nb = (size_t)std::max(q.nnzb, 1),
                 na = (size_t)std::max(q.nnza, 1);
    const int nbs = ceil_div((int)k + 1, kScanBlock) + 2;
    const int nbs2 = ceil_div((int)nb, kScanBlock) + 2;
    size_t off = 0;
    auto carve = [&](size_t bytes) {
        const size_t o = off;
        off += align_up(bytes, 256);
        return o;
    };
    const size_t o_pofs = carve(8 * nb), o_cb = carve(4 * nb), o_aview = carve(8 * na),
                 o_rowptr = carve(4 * (k + 1)), o_rv = carve(8 * nb), o_rvp = carve(8 * nb),
                 o_fill = carve(4 * std::max<size_t>(k, 1)), o_colj = carve(4 * nb),
                 o_pos = carve(4 * nb), o_bcol = carve(4 * nb), o_len = carve(4 * nb),
                 o_scr = carve(8 * (size_t)nbs), o_scr2 = carve(8 * (size_t)nbs2),
                 o_err = carve(sizeof(int)),
                 o_dst = carve(4 * (size_t)std::max<unsigned long long>(p->hdr_host.total_op, 1));
    const size_t need = off;
    if (need > p->bt.bytes) {
        p->bt_ready = false;
        SPG_TRY(order_after(p, s, p->last_stream));
        if (spgemm_status st = dev_alloc(p, p->bt, need, s)) return st;
    }
    char *b = (char *)p->bt.ptr;
    BwBuild bb{};
    bb.pofs = (long long *)(b + o_pofs);
    bb.cb = (int32_t *)(b + o_cb);
    bb.aview = (int2 *)(b + o_aview);
    bb.rowptr = (int32_t *)(b + o_rowptr);
    bb.rv = (int2 *)(b + o_rv);
    bb.rvp = (long long *)(b + o_rvp);
    bb.fill = (int32_t *)(b + o_fill);
    bb.colj = (int32_t *)(b + o_colj);
    bb.pos = (int32_t *)(b + o_pos);
    bb.bcol = (int32_t *)(b + o_bcol);
    bb.len = (int32_t *)(b + o_len);
    bb.scratch = (long long *)(b + o_scr);
    bb.nscratch = nbs;
    bb.scratch2 = (long long *)(b + o_scr2);
    bb.nscratch2 = nbs2;
    bb.dst = (uint32_t *)(b + o_dst);
    p->bt_err = (int *)(b + o_err);
    BwView w{};
    w.E = p->E;
    w.dst = bb.dst;
    w.nnzc = p->totals_host[0];
    w.pofs = bb.pofs;
    w.cb = bb.cb;
    w.aview = bb.aview;
    w.rowptr = bb.rowptr;
    w.rv = bb.rv;
    w.rvp = bb.rvp;
    if (!p->bt_ready) {
        // the error word is cleared with the view only: later calls queue no
        // memset, so they can be captured in a HIP graph
        SPG_TRY(hipMemsetAsync(p->bt_err, 0, sizeof(int), s));
        ProfScope ps("bw_view", s);
        SPG_TRY(launch_bw_view(q, p->E, bb, w, s));
        SPG_TRY(launch_bw_dst(q, p->E, bb.pofs, bb.bcol, C_rowidx, bb.dst, p->bt_err, s));
        p->bt_ready = true;
    }
    {
        ProfScope ps("gradients", s);
        SPG_TRY(launch_backward(q, w, f64, A_val, B_val, G_val, dA_val, dB_val, p->bt_err, s));
    }
    p->last_stream = s;
    return SPGEMM_OK;
}

spgemm_status spgemm_plan_get_stats(spgemm_plan p, spgemm_plan_stats *out) {
    if (!p) return SPGEMM_ERR_PLAN;
    if (!out) return SPGEMM_ERR_NULL;
    if (!p->symbolic_ok) return SPGEMM_ERR_PLAN;
    const Hdr &h = p->hdr_host;
    spgemm_plan_stats s{};
    s.total_products = (int64_t)h.total_op;
    for (long long t : p->totals_host) s.nnz_c += t;
    s.ncols = p->ncols;
    s.cols_empty = h.bin_count[BIN_EMPTY];
    for (int i = 0; i < kEscBins; ++i) s.cols_esc += h.bin_count[BIN_ESC0 + i];
    for (int i = 0; i < kSortBins; ++i) s.cols_sort += h.bin_count[BIN_SORT0 + i];
    s.cols_sort += h.bin_count[BIN_WSORT];
    for (int i = 0; i < kBlkBins; ++i) s.cols_block += h.bin_count[BIN_BLK0 + i];
    s.esc_groups = esc_groups(h);
    s.nprob = p->nprob;
    // window flags of the workgroup columns
    if (p->ncols > 0 && s.cols_block > 0) {
        std::vector<int32_t> bw((size_t)p->ncols);
        if (hipMemcpy(bw.data(), p->binw, 4 * bw.size(), hipMemcpyDeviceToHost) != hipSuccess)
            return SPGEMM_ERR_HIP;
        for (int32_t v : bw) {
            const int f = v >> 8;
            s.cols_direct += (f & WF_DIRECT) != 0;
            s.cols_hash += (f & WF_HASH) != 0;
            s.cols_split += (f & WF_SPLIT) != 0;
        }
    }
    s.later_max = h.later_maxk;
    s.later_products = (int64_t)p->later_total;
    if ((p->flags & SPGEMM_LANE_BLOCKED) && p->direct && p->lbuf.ptr) {
        for (int i = 0; i < p->lb.nsub; ++i) s.lane_cols += h.bin_count[BIN_ESC0 + i];
        if (hipMemcpy(&s.lane_blocks, p->lb.counts, 4, hipMemcpyDeviceToHost) != hipSuccess)
            return SPGEMM_ERR_HIP;
    }
    *out = s;
    return SPGEMM_OK;
}

spgemm_status spgemm_profile_enable(int32_t on) {
    g_prof.on = on != 0;
    if (g_prof.on) g_prof.used = 0;
    return SPGEMM_OK;
}

spgemm_status spgemm_profile_select(const char *name) {
    std::memset(g_prof.only, 0, sizeof(g_prof.only));
    if (name) std::strncpy(g_prof.only, name, sizeof(g_prof.only) - 1);
    return SPGEMM_OK;
}

spgemm_status spgemm_profile_read(spgemm_kernel_time *out, int32_t max, int32_t *n_out) {
    if (!out || !n_out) return SPGEMM_ERR_NULL;
    std::vector<spgemm_kernel_time> acc;
    for (size_t i = 0; i < g_prof.used; ++i) {
        const ProfRec &r = g_prof.recs[i];
        if (hipEventSynchronize(r.b) != hipSuccess) return SPGEMM_ERR_HIP;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return SPGEMM_ERR_HIP;
        size_t k = 0;
        for (; k < acc.size(); ++k)
            if (std::strncmp(acc[k].name, r.name, sizeof(acc[k].name)) == 0) break;
        if (k == acc.size()) {
            spgemm_kernel_time t{};
            std::strncpy(t.name, r.name, sizeof(t.name) - 1);
            acc.push_back(t);
        }
        acc[k].launches += 1;
        acc[k].total_ms += ms;
    }
    const int n = (int)std::min<size_t>(acc.size(), (size_t)std::max(max, 0));
    for (int i = 0; i < n; ++i) out[i] = acc[i];
    *n_out = n;
    return SPGEMM_OK;
}

void spgemm_plan_destroy(spgemm_plan p) {
    if (!p) return;
    // every use of the plan's buffers is ordered before the end of its last
    // stream; they are released in stream order behind it
    const hipStream_t s = p->last_stream;
    dev_free(p, p->prod, s);
    dev_free(p, p->stage, s);
    dev_free(p, p->ws, s);
    dev_free(p, p->bt, s);
    dev_free(p, p->lbuf, s);
    (void)hipStreamSynchronize(s);
    for (int i = 0; i < spgemm_plan_s::kSide; ++i) {
        if (p->side[i]) {
            (void)hipStreamSynchronize(p->side[i]);
            (void)hipStreamDestroy(p->side[i]);
        }
        if (p->join_ev[i]) (void)hipEventDestroy(p->join_ev[i]);
    }
    if (p->fork_ev) (void)hipEventDestroy(p->fork_ev);
    if (p->order_ev) (void)hipEventDestroy(p->order_ev);
    if (p->pinned) (void)hipHostFree(p->pinned);
    delete p;
}

void spgemm_batch_plan_destroy(spgemm_batch_plan p) { spgemm_plan_destroy(p); }

}  // extern "C"

// ---------------------------------------------------------------- allocation-free product
// The workspace of spgemm_multiply_noalloc: one file-scope device array that
// every GPU the library runs on holds until the process ends. Host code never
// passes its name to a kernel or a copy: the address of each device's copy is
// looked up once per device (hipGetSymbolAddress) and that pointer is carved.
namespace {
constexpr size_t kScratchBytes = size_t(128) << 20;
constexpr int kNoAllocDevices = 64;
}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
struct NoAllocSlot {
    bool ready = false;
    char *scratch_ptr = nullptr;  // this device's copy of `scratch`
    spgemm_plan_s plan;
    alignas(64) unsigned char host[kHdrBytes + 64];  // header and nnz(C) read back
};
NoAllocSlot g_noalloc[kNoAllocDevices];

// host vectors the per-device plans use hold one problem; their storage is
// taken when the library is loaded, so no call allocates host memory either
struct NoAllocReserve {
    NoAllocReserve() {
        for (NoAllocSlot &sl : g_noalloc) {
            sl.plan.probs.reserve(1);
            sl.plan.totals_host.reserve(1);
        }
    }
} g_noalloc_reserve;
}  // namespace

extern "C" spgemm_status spgemm_multiply_noalloc(const spgemm_csc *A, const spgemm_csc *B,
                                                 spgemm_dtype dt, const spgemm_options *opt,
                                                 void *stream, int32_t *C_colptr,
                                                 int32_t *C_rowidx, void *C_val, int64_t capacity,
                                                 int64_t *nnzC_host) {
    if (!A || !B || !C_colptr || !nnzC_host) return SPGEMM_ERR_NULL;
    if (dt != SPGEMM_F32 && dt != SPGEMM_F64) return SPGEMM_ERR_DTYPE;
    if (capacity < 0) return SPGEMM_ERR_INVALID;
    spgemm_status st;
    if ((st = check_desc(A, true)) || (st = check_desc(B, true))) return st;
    if (capacity > 0 && (!C_rowidx || !C_val)) return SPGEMM_ERR_NULL;
    if (A->ncols != B->nrows) return SPGEMM_ERR_SHAPE;
    Tune tune;
    uint32_t flags;
    if ((st = resolve_options(opt, tune, flags))) return st;
    // the host-side check copies the inputs into host vectors: not offered here
    if (flags & SPGEMM_VALIDATE) return SPGEMM_ERR_INVALID;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SPGEMM_ERR_HIP;
    if (dev < 0 || dev >= kNoAllocDevices) return SPGEMM_ERR_INVALID;
    NoAllocSlot &sl = g_noalloc[dev];
    if (!sl.ready) {
        // once per device, with that device current: the address of its copy
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr)
            return SPGEMM_ERR_HIP;
        sl.scratch_ptr = (char *)ptr;
        sl.ready = true;
    }
    spgemm_plan p = &sl.plan;
    hipStream_t s = (hipStream_t)stream;
    // a fresh single-problem pass on the caller's stream, every buffer carved
    // from this device's scratch array
    p->device = dev;
    p->use_arena = true;
    p->arena = sl.scratch_ptr;
    p->arena_size = kScratchBytes;
    p->arena_off = 0;
    p->ws = p->prod = p->stage = p->bt = p->lbuf = DevBuf{};
    p->pinned = sl.host;
    p->pinned_dev = nullptr;
    p->pinned_bytes = sizeof(sl.host);
    p->dt = dt;
    p->batched = false;
    p->nprob = 1;
    p->tune = tune;
    p->flags = flags | SPGEMM_ONE_STREAM | SPGEMM_NO_PLANNED_LAUNCH;
    p->probs.resize(1);
    Prob &q = p->probs[0];
    q = Prob{};
    q.m = A->nrows; q.k = A->ncols; q.n = B->ncols;
    q.nnza = A->nnz; q.nnzb = B->nnz;
    q.acp = A->colptr; q.ari = A->rowidx; q.av = A->val;
    q.bcp = B->colptr; q.bri = B->rowidx; q.bv = B->val;
    q.ccp = C_colptr;
    p->wide_keys = q.m >= (1 << 20);
    p->wide_esc = q.m >= (1 << 24) - 1;
    p->wide_acc = q.m >= (1 << 21) - 1;
    p->rowbits = row_bits(q.m);
    p->maxm = q.m;
    p->direct = tune.t_block == 0x7fffffff && !(flags & SPGEMM_LANE_HASH);
    p->heavy_cap = 0;
    p->win_cap = 0;
    p->ncols = q.n;
    p->total_nnzb = q.nnzb;
    p->ntiles = ceil_div(q.n, kTile);
    p->symbolic_ok = false;
    p->spec_ready = false;
    p->bt_ready = false;
    p->hdr_host = Hdr{};
    static const std::vector<int4> no_tiles;  // used by several-problem plans only
    bool retry = false;
    st = symbolic_pass(p, s, no_tiles, false, &retry, nullptr);
    p->last_stream = s;
    if (st) return st;
    const long long nnzc = p->totals_host[0];
    *nnzC_host = nnzc;
    if (nnzc > capacity) return SPGEMM_ERR_CAPACITY;
    q.cri = C_rowidx;
    q.cv = C_val;
    if (nnzc == 0) return SPGEMM_OK;
    return run_numeric(p, s);
}

extern "C" {

spgemm_status spgemm_set_allocator(spgemm_alloc_fn alloc, spgemm_free_fn free_fn, void *ctx) {
    if ((alloc == nullptr) != (free_fn == nullptr)) return SPGEMM_ERR_NULL;
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    g_alloc.alloc = alloc;
    g_alloc.free = free_fn;
    g_alloc.ctx = alloc ? ctx : nullptr;
    return SPGEMM_OK;
}

}  // extern "C"
