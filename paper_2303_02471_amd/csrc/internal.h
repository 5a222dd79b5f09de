// Internal definitions shared by the HIP kernels and the host planner of the
// column-wise sparse product C = A x B (CSC, Section 2.1 of the paper).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace spg {

constexpr int kWave = 64;

// ---------------------------------------------------------------- bins
// A column's accumulator is chosen from its product count Op_j (Section 3.1):
//   EMPTY      Op_j == 0: no output entries
//   ESC_i      Op_j <= 4 << i: wavefront sort-merge (Section 4), 64 >> i
//              columns per wavefront group (at most 256 products)
//   SORT_i     Op_j <= 512 << i (and <= t_sort): workgroup sort-merge, one
//              column per workgroup of 128 << i threads
//   DENSE      dense LDS accumulator over all rows (SPA, Section 2.2)
//   HASH_S/L/XL LDS hash table per row window (HASH, Section 3.2); the bins
//              differ only in the largest table they hold, so the smaller ones
//              run with a smaller LDS footprint (more workgroups per CU)
enum Bin : int {
    BIN_EMPTY = 0,
    BIN_ESC0 = 1,  // Op <= 4
    BIN_ESC6 = 7,  // Op <= 256
    BIN_SORT0 = 8, // Op <= 512
    BIN_SORT3 = 11, // Op <= 4096
    BIN_DENSE = 12,
    BIN_HASH_S = 13,
    BIN_HASH_L = 14,
    BIN_HASH_XL = 15,
    NBINS = 16
};
constexpr int kHashBins = 3;
constexpr int kEscBins = 7;
constexpr int kSortBins = 4;
constexpr int kSortMax = 4096;        // products per workgroup sort
constexpr int kProdTile = 1024;       // products per product-balanced tile
constexpr int kOrderMax = 2048;       // largest column the tiles write in output order
// every column of the sort bins below the largest one is written in output order
static_assert(kOrderMax == (512 << (kSortBins - 2)), "ordered columns end below the last sort bin");
constexpr int kEscMaxProducts = 256;  // products per wavefront group

// dense accumulator: rows per LDS slice
constexpr int kDenseRows = 4096;
// hash accumulator: largest table of the small, large and extra-large class,
// smallest table, and the probe overrun area behind a table of h slots
constexpr int kHashMaxS = 1024;
constexpr int kHashMaxL = 4096;
constexpr int kHashMax = 8192;
constexpr int kHashMin = 64;
__host__ __device__ constexpr int hash_class(int h) { return h <= kHashMaxS ? 0 : (h <= kHashMaxL ? 1 : 2); }
__host__ __device__ constexpr int hash_pad(int h) { return h >= 1024 ? 256 : h / 4; }
constexpr int kBlock = 256;
// columns per classification tile
constexpr int kTile = 512;
// row windows per hash column (a window holding more distinct rows than its
// table splits itself)
constexpr int kMaxWindows = 4096;

// error bits gathered on the device
enum ErrBits : int {
    ERR_CSC = 1,        // malformed input seen by a kernel
    ERR_OPOVF = 2,      // a column's product count exceeds INT32_MAX
    ERR_ITEMCAP = 4,    // hash row windows exceed the workspace capacity
    ERR_NNZOVF = 8,     // nnz(C) of a problem exceeds INT32_MAX
    ERR_GROUP = 16      // a wavefront group exceeded its bounds (inputs changed)
};

// One problem of a (possibly single-problem) batch. All pointers are device
// pointers. Column j of this problem is global column col0 + j.
struct Prob {
    int32_t m, k, n, col0;
    int32_t nnza, nnzb;
    long long ebase;  // offset of this problem's stored B entries in KArgs::E
    const int32_t *acp, *ari;
    const void *av;
    const int32_t *bcp, *bri;
    const void *bv;
    int32_t *ccp, *cri;
    void *cv;
};

// Device header written by the planning kernels.
struct Hdr {
    int32_t bin_count[NBINS];
    int32_t bin_cursor[NBINS];
    int32_t item_count[kHashBins];    // row windows (work items) per hash bin
    int32_t pad0;
    unsigned long long hash_cursor[kHashBins];  // (items << 32) | columns placed, per hash bin
    int32_t err;
    int32_t pad;
    unsigned long long total_op;
    unsigned long long list_products;  // products of the dense and hash columns
    unsigned long long later_count;    // products that are not the first of their output entry
    int32_t later_maxk;                // largest occurrence index k of any product
    int32_t pad2;
};

// Resolved tuning values.
struct Tune {
    int32_t esc_bins;   // number of ESC sub-bins in use, 1..7 (t_esc = 4 << (esc_bins-1))
    int32_t t_sort;     // largest product count of a workgroup-sort column (<= kSortMax)
    int32_t t_dense;
    int32_t dense_rows;
    int32_t hash_cap;
};

// Kernel arguments common to all planning / accumulation kernels.
struct KArgs {
    Prob single;            // used when nprob == 1
    const Prob *table;      // device table when nprob > 1
    const int32_t *col0s;   // device [nprob + 1] global column offsets (nprob > 1)
    int32_t nprob;
    int32_t ncols;          // total columns over all problems
    int32_t ntiles;
    int32_t item_cap;
    const int4 *tiles;      // (pid, j0, j1, 0) when nprob > 1
    Tune tune;
    Hdr *hdr;
    int32_t *op;            // [ncols]
    int32_t *binw;          // [ncols] bin | (windows << 8)
    int4 *binlist;          // [ncols] (global column, first stored B entry, B entries, 0),
                            // grouped by bin
    int32_t *gnnz;          // [ncols]
    int4 *items;            // [item_cap] (global column, bin-list position, first B entry,
                            // B entries) of every hash row window, hash bins in order; the
                            // windows of one column are consecutive from colitem[column]
    int32_t *itemcnt;       // [item_cap] distinct rows of every hash row window
    int32_t *itemoff;       // [item_cap] distinct rows of the column's earlier windows
    int32_t *colitem;       // [ncols] first work item of every hash column (by global column)
    int2 *E;                // [sum of nnz(B)] (A column start, A column length) of every
                            // stored B entry, written by the classification
    // Product space: the products of all columns in column order (problems in
    // order), each column's products in the order Algorithm 1 meets them:
    // stored B entries in storage order, then the rows of the selected A
    // column in storage order.
    long long *colprod;     // [ncols + 1] first product of every global column
    int32_t *prow;          // [products] row of every product (written once by the expansion)
    uint32_t *dst;          // [products] destination of every product (see below)
    // Output order of the columns with at most kSortMax products and no row
    // windows: perm[colprod[g] + r] = position in the column's product list of
    // the first product of the column's output entry r, crow[colprod[g] + r] =
    // the row of that entry.
    int32_t *perm;          // [products]
    int32_t *crow;          // [products]
    // Product-balanced tiles: tile t holds the columns whose first product
    // lies in [t * kProdTile, (t + 1) * kProdTile).
    int32_t *tilestart;     // [nptiles + 1] first global column of every tile
    int32_t nptiles;
    // Products that are not the first of their output entry ("later"
    // products), in a compact list: occurrence index k >= 1 and output rank
    // (symbolic), and the output position, problem and value staged by the
    // numeric phase.
    long long later_cap;
    int32_t *lk;            // [later_cap]
    int32_t *lr;            // [later_cap] rank of the output row (as in dst)
    int32_t *lo;            // [later count]
    int32_t *lpid;          // [later count]
    void *lv;               // [later count] values (V)
};

// Destination code of a product: the rank of its output row inside its
// column (for a hash column split into row windows: inside its window), or,
// for a later product, kDstLater | its index in the later list.
constexpr uint32_t kDstLater = 0x80000000u;

__host__ __device__ inline int ceil_div(int a, int b) { return (a + b - 1) / b; }

__device__ __forceinline__ int find_prob(const KArgs &a, int g) {
    if (a.nprob == 1) return 0;
    int lo = 0, hi = a.nprob;  // last p with col0s[p] <= g
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (a.col0s[mid] <= g) lo = mid;
        else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ Prob get_prob(const KArgs &a, int pid) {
    return a.nprob == 1 ? a.single : a.table[pid];
}

// Number of hash row windows of a column with `op` products (at most
// kMaxWindows; a window holding too many distinct rows splits itself).
__host__ __device__ inline int hash_windows(int op, int cap) {
    const int w = op <= cap ? 1 : ceil_div(op, cap);
    return w < kMaxWindows ? w : kMaxWindows;
}

// Row window [lo(w), lo(w+1)) of w in [0, W) over m rows, and the window of a row.
__host__ __device__ inline int window_lo(int w, int W, int m) {
    return (int)(((long long)w * m) / W);
}
__host__ __device__ inline int window_of(int row, int W, int m) {
    int w = (int)(((long long)row * W) / (m > 0 ? m : 1));
    if (w >= W) w = W - 1;
    while (w + 1 < W && window_lo(w + 1, W, m) <= row) ++w;
    while (w > 0 && window_lo(w, W, m) > row) --w;
    return w;
}

// Table size of one hash row window: a power of two at least twice the
// planned distinct rows (load factor <= 1/2), within [kHashMin, kHashMax].
__host__ __device__ inline int hash_table_size(int op, int windows) {
    int per = ceil_div(op, windows);
    int h = kHashMin;
    while (h < 2 * per && h < kHashMax) h <<= 1;
    return h;
}

// ---------------------------------------------------------------- launchers
// Each returns hipSuccess or the launch error.
hipError_t launch_classify(const KArgs &a, hipStream_t s);
hipError_t launch_place(const KArgs &a, hipStream_t s);
hipError_t launch_esc(const KArgs &a, int grid, hipStream_t s);
// workgroup sort of sort bin `cls`; wide: 64-bit keys (rows beyond 20 bits)
hipError_t launch_sort(const KArgs &a, int cls, bool wide, int grid, hipStream_t s);
// mode: dense, or one of the three hash table classes
enum WinMode : int { WIN_DENSE = 0, WIN_HASH_S = 1, WIN_HASH_L = 2, WIN_HASH_XL = 3 };
hipError_t launch_window(const KArgs &a, int mode, int grid, hipStream_t s);
hipError_t launch_scan(const KArgs &a, long long *gcp, long long *bsum, int nblk,
                       long long *totals, hipStream_t s);
// first product of every global column (colprod) and first column of every
// product-balanced tile (tilestart); bsum holds nbsum scan partials
hipError_t launch_prod_offsets(const KArgs &a, long long *bsum, int nbsum, hipStream_t s);
// row of every product (prow), one workgroup per product-balanced tile
hipError_t launch_expand(const KArgs &a, hipStream_t s);
// numeric phase of the columns with an output order (one workgroup per
// product-balanced tile) and of the others (one workgroup per column from
// bin-list position `first`, `nbig` positions): first products written to
// their output entries, later products staged
hipError_t launch_numeric(const KArgs &a, bool f64, hipStream_t s);
hipError_t launch_numeric_big(const KArgs &a, bool f64, int first, int nbig, hipStream_t s);
// adds the staged later products of occurrence index k (n of them listed)
hipError_t launch_layer(const KArgs &a, bool f64, int k, long long n, hipStream_t s);
hipError_t launch_btranspose(const Prob &p, int32_t *rowptr, int32_t *fill, int32_t *colj,
                             int32_t *pos, long long *scratch, int nscratch, hipStream_t s);
hipError_t launch_backward(const Prob &p, bool f64, const void *av, const void *bv,
                           const int32_t *cri, const void *gv, void *da, void *db,
                           const int32_t *rowptr, const int32_t *colj, const int32_t *pos,
                           int *err, hipStream_t s);
hipError_t launch_scan_i32(const int32_t *in, int n, long long *bsum, int nbsum, int32_t *out,
                           hipStream_t s);

constexpr int kScanBlock = 1024;  // elements per scan block

}  // namespace spg
