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
//   ESC_i      Op_j <= 4 << i (and <= t_esc): wavefront sort-merge (Section 4),
//              64 >> i columns per wavefront group (at most 256 products)
//   SORT_i     Op_j <= 512 << i: workgroup sort-merge, one column per
//              workgroup of 128 << i threads
//   WSORT      Op_j > 4096: the same sort over row windows of the column, one
//              workgroup per column taking the windows in row order
//   BLK_c      Op_j > t_block instead of SORT / WSORT (an option): one
//              workgroup per column with an LDS table over
//              row windows -- a direct-indexed SPA (Section 2.2) when the
//              window's row span fits, else an order-preserving hash table
//              with linear probing (Section 3.2) sized from Op_j (its size
//              adaptation). The classes differ in workgroup size and LDS
//              footprint: Op_j <= 512, 1024, 2048, 4096, and above.
enum Bin : int {
    BIN_EMPTY = 0,
    BIN_ESC0 = 1,   // Op <= 4
    BIN_ESC6 = 7,   // Op <= 256
    BIN_SORT0 = 8,  // Op <= 512
    BIN_SORT2 = 10, // Op <= 2048
    BIN_SORT3 = 11, // Op <= 4096
    BIN_WSORT = 12, // Op > 4096
    BIN_BLK0 = 13,  // Op <= 512
    BIN_BLK4 = 17,  // Op > 4096
    NBINS = 18
};
constexpr int kEscBins = 7;
constexpr unsigned long long kSmallProducts = 1u << 20;  // below: accumulators on one stream
constexpr int kLaneSubBins = 2;  // wavefront sub-bins below this: one column per lane
constexpr int kEscSide0 = 5;  // wavefront sub-bins below this (at most 64 products) share one
                              // accumulator stream, the larger ones the one-column waves' stream
constexpr int kSortBins = 4;
constexpr int kBlkBins = 5;
constexpr int kSortMax = 4096;        // products per workgroup sort
constexpr int kProdTile = 2048;       // products per product-balanced tile
constexpr int kEscMaxProducts = 256;  // products per wavefront group
constexpr int kChunkB = 256;          // stored B entries per chunk of a split column

__host__ __device__ constexpr int blk_class(int op) {
    return op <= 512 ? 0 : (op <= 1024 ? 1 : (op <= 2048 ? 2 : (op <= 4096 ? 3 : 4)));
}
constexpr int kBlock = 256;
// columns per classification tile
constexpr int kTile = 512;

// error bits gathered on the device
enum ErrBits : int {
    ERR_CSC = 1,        // malformed input seen by a kernel
    ERR_OPOVF = 2,      // a column's product count exceeds INT32_MAX
    ERR_NNZOVF = 8,     // nnz(C) of a problem exceeds INT32_MAX
    ERR_GROUP = 16,     // a work item exceeded its planned bounds (inputs changed)
    ERR_RETRY = 32      // a launch planned from an earlier call met other sizes: the
                        // product-space kernels did nothing, the host redoes the phase
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
    int32_t err;
    int32_t later_maxk;                // largest occurrence index k of any product
    int32_t big_chunks;                // most kChunkB-entry chunks of a column above t_split
    int32_t cap_over;                  // nnz(C) exceeds the output capacity of a one-call product
    unsigned long long total_op;
    unsigned long long heavy_prod;     // products of the heavy columns (bins SORT3, WSORT)
    int32_t heavy_win;                 // row windows of the heavy columns
    int32_t pad_;
};

// binw[g] = bin | (window flags << 8); the workgroup accumulator records how
// it accumulated the column's row windows
enum WinFlags : int { WF_DIRECT = 1, WF_HASH = 2, WF_SPLIT = 4 };

// Resolved tuning values.
struct Tune {
    int32_t esc_bins;    // number of ESC sub-bins in use, 1..7 (t_esc = 4 << (esc_bins-1))
    int32_t t_dense;     // smallest product count of a column that may use direct indexing
    int32_t dense_rows;  // largest row span of a direct-indexed window (0: table capacity)
    int32_t hash_cap;    // planned distinct rows per row window (0: table capacity / 2)
    int32_t t_split;     // columns with more products are split over several numeric workgroups
    int32_t t_block;     // columns with more products go to the workgroup hash accumulator
                         // (instead of the sort-merge ones)
    int32_t t_lane;      // lane-per-column blocks: columns of at most t_lane products
    int32_t b_min, b_max;  // block sizes of the Blocking Algorithm
};

// Kernel arguments common to all planning / accumulation kernels.
struct KArgs {
    Prob single;            // used when nprob == 1
    const Prob *table;      // device table when nprob > 1
    const int32_t *col0s;   // device [nprob + 1] global column offsets (nprob > 1)
    int32_t nprob;
    int32_t ncols;          // total columns over all problems
    int32_t ntiles;
    const int4 *tiles;      // (pid, j0, j1, 0) when nprob > 1
    // per classification tile: the tile's column count of every bin (then the
    // tile's first position inside the bin), its products and the most
    // chunks of one of its columns above t_split
    int32_t *th;            // [ntiles * NBINS]
    long long *ttot;        // [ntiles]
    int32_t *tmax;          // [ntiles]
    Tune tune;
    // A symbolic launch planned before the sizes are read back (from the
    // previous call on the plan) covers the bins in spec_mask with product
    // space for spec_total products; spec_total < 0 when the launch follows
    // the read-back.
    long long spec_total;
    unsigned spec_mask;
    Hdr *hdr;
    int32_t *op;            // [ncols]
    int32_t *binw;          // [ncols] bin of every global column, window flags
    int4 *binlist;          // [ncols] (global column, first stored B entry, B entries, Op_j),
                            // grouped by bin
    int32_t *gnnz;          // [ncols]
    int2 *E;                // [sum of nnz(B)] (A column start, A column length) of every
                            // stored B entry, written by the classification
    // Product space: the products of all columns in column order (problems in
    // order), each column's products in the order Algorithm 1 meets them:
    // stored B entries in storage order, then the rows of the selected A
    // column in storage order.
    long long *colprod;     // [ncols + 1] first product of every global column
    int32_t *prow;          // [products] row of every product (written once by the expansion)
    uint32_t *dst;          // [products] destination of every product (see below)
    // Product-balanced tiles: tile t holds the columns whose first product
    // lies in [t * kProdTile, (t + 1) * kProdTile).
    int32_t *tilestart;     // [nptiles + 1] first global column of every tile
    int32_t nptiles;
    long long prod_cap;     // products the product-space arrays hold: the expansion and
                            // the numeric phase never address beyond (ERR_GROUP instead)
    // Products that are not the first of their output entry ("later"
    // products). The symbolic phase gives each its occurrence index k >= 1
    // and its index among the later products of its column (both stored at
    // the product's position). Column g has Op_g - nnz(C(:,g)) of them, so
    // the later products of all columns form a compact list in which column
    // g's start at colprod[g] - (entries of C before column g); the numeric
    // phase stages there the output position, problem, value and k of each.
    int32_t *lk;            // [products] k of every later product
    int32_t *lr;            // [products] index of every later product in its column
    const long long *gcp;   // [ncols + 1] entries of C before every global column (nprob > 1)
    long long later_n;      // length of the compact list (numeric phase)
    long long out_cap;      // entries the caller's C arrays hold (single problem; else no limit)
    int32_t *lo;            // [later_n] output position
    int32_t *lpid;          // [later_n] problem
    int32_t *lkc;           // [later_n] occurrence index k
    void *lv;               // [later_n] value (V)
    // Heavy columns of the direct-gather accumulators (bins SORT3 and WSORT,
    // adjacent in the bin list, position li among them): first product in the
    // heavy scratch, first row window, and the scratch itself.
    long long *hoff;        // [heavy columns + 1]
    int32_t *wbase;         // [heavy columns + 1]
    int32_t *wcnt;          // [windows] output entries of every window (symbolic phase)
    int32_t *winmap;        // [windows] heavy column (position li) of every window
    int32_t *hrow;          // [heavy products] row of every product of a heavy column
    void *hval;             // [heavy products] its value A(i,k) B(k,j) (numeric phase, V)
    uint32_t *hperm;        // [2 heavy_cap] product indices of the radix sort (SPGEMM_RADIX_ESC)
    long long heavy_cap;    // heavy products / windows the scratch holds: a launch planned
    int32_t win_cap;        // from an earlier call that finds more is redone
    // Numeric phase run at the column positions of the plan's previous
    // structure (single problem, before this call's counts are scanned): it
    // also records every column's entry count, and a count that differs
    // from the previous structure asks for a redo (ERR_RETRY).
    int32_t spec_fill;
};

// Destination code of a product: the rank of its output row inside its
// column, with kDstLater set when the product is not the first of its entry.
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

// ---------------------------------------------------------------- launchers
// Each returns hipSuccess or the launch error.
hipError_t launch_classify(const KArgs &a, hipStream_t s);
// bin counts, product total and largest chunk count from the tile tallies;
// per-tile positions inside every bin
hipError_t launch_tally(const KArgs &a, hipStream_t s);
hipError_t launch_place(const KArgs &a, hipStream_t s);
// wavefront groups of ESC sub-bin `sub`; wide: 64-bit keys (rows of 2^24 - 1 and more)
hipError_t launch_esc(const KArgs &a, bool wide, int sub, int groups, hipStream_t s);
// every sub-bin in one launch; groups[i] wavefront groups of sub-bin i (0: none)
hipError_t launch_esc_all(const KArgs &a, bool wide, const int *groups, hipStream_t s);
// lane-per-column hash accumulator over ESC sub-bin `sub` (at most 64 products,
// ncols columns): the same outputs as launch_esc
hipError_t launch_lane(const KArgs &a, int sub, int ncols, hipStream_t s);
constexpr int kLaneMaxSub = 4;  // sub-bins 0..4 (up to 64 products) may take it
// workgroup sort of sort bin `cls` (n columns); wide: 64-bit keys (rows beyond 20 bits)
hipError_t launch_sort(const KArgs &a, int cls, bool wide, int n, hipStream_t s);
// windowed workgroup sort (columns from the device header; any grid covers them)
hipError_t launch_wsort(const KArgs &a, bool wide, int grid, hipStream_t s);
// workgroup hash accumulator of block class `cls` (columns and their bin-list
// positions from the device header; any grid covers them)
hipError_t launch_block(const KArgs &a, int cls, int grid, hipStream_t s);
hipError_t launch_scan(const KArgs &a, long long *gcp, long long *bsum, int nblk,
                       long long *totals, hipStream_t s);
// first product of every global column (colprod) and first column of every
// product-balanced tile (tilestart); bsum holds nbsum scan partials
hipError_t launch_prod_offsets(const KArgs &a, long long *bsum, int nbsum, hipStream_t s);
// row of every product (prow), one workgroup per product-balanced tile
hipError_t launch_expand(const KArgs &a, hipStream_t s);
// numeric phase, one launch: the columns of at most t_split products by
// product-balanced tiles (one workgroup per tile), the larger ones (listed
// from bin-list position `first`, `nbig` of them, with at most `maxchunks`
// chunks of kChunkB stored B entries) by one workgroup per chunk; first
// products are written to their output entries, later products staged
hipError_t launch_numeric(const KArgs &a, bool f64, int first, int nbig, int maxchunks,
                          hipStream_t s);
// adds the staged later products of occurrence index k (n of them listed)
hipError_t launch_layer(const KArgs &a, bool f64, int k, long long n, hipStream_t s);
// adds every staged later product in one launch; needs later lists in sorted
// key order (no hash-accumulator columns)
hipError_t launch_later_runs(const KArgs &a, bool f64, long long n, hipStream_t s);
// Direct-gather accumulators (no per-product arrays between the phases).
// fill = false: distinct rows per column (gnnz; window counts of heavy
// columns); fill = true: rows and values of C. wide: 64-bit keys (rows of
// 2^21 - 1 and more).
int wave_bin_items(int bin, int ncols);
hipError_t launch_acc_wave(const KArgs &a, int bin, int items, bool wide, bool fill, bool f64,
                           hipStream_t s);
// offsets and windows of the heavy columns; totals to the header
hipError_t launch_heavy_plan(const KArgs &a, hipStream_t s);
// global ESC with radix sort over groups of heavy columns (after the heavy
// expansion); rowbits: bits of the largest row index
hipError_t launch_esc_radix(const KArgs &a, long long heavy_products, int rowbits, bool fill,
                            bool f64, hipStream_t s);
// expansion of the ncols heavy columns and their nwin windows
// Lane-per-column blocks of the sorted light columns (SPGEMM_LANE_BLOCKED)
constexpr int kLbMaxT = 64;                  // largest t (products of a lane column)
constexpr int kLbMaxDesc = 4 * kLbMaxT + 8;  // block descriptors of one plan
constexpr int kSparsMaxRows = 4096;          // rows of a SPARS lane accumulator
struct LbArgs {
    int32_t t;          // lane columns: Op_j <= t (the first nsub ESC sub-bins)
    int32_t b_min, b_max;
    int32_t nsub;
    int32_t mslab;      // rows of a SPARS value slab (largest m)
    int32_t *hist;      // [t + 1] lane columns per Op value (zero between calls)
    int32_t *pos;       // [t + 1] next position of every Op value in the sorted order
    int32_t *counts;    // [2] blocks, descriptors
    int4 *desc;         // [kLbMaxDesc] (first position, blocks, block size, first block)
    int4 *sorted;       // [ncap] bin entries by decreasing Op
    int32_t ncap;       // entries `sorted` holds (the plan's columns)
    void *dense;        // value slabs, one per wavefront of the block launch
};
hipError_t launch_lane_blocked(const KArgs &a, const LbArgs &lb, int ncols_hint, int grid_cap,
                               bool spars, bool fill, bool f64, hipStream_t s);

// heavy columns: windows, or (radix) the global radix ESC; heavy_products and
// rowbits size the radix launch
// part 0 .. heavy_parts(radix) - 1 of the heavy columns' launches, in order;
// a launch whose heavy plan ran in it (planned) starts at heavy_first_part
int heavy_parts(bool radix);
int heavy_first_part(bool radix, bool planned);
hipError_t launch_heavy(const KArgs &a, int ncols, int nwin, bool wide, bool fill, bool f64,
                        hipStream_t s, bool radix, long long heavy_products, int rowbits,
                        int part);
inline int row_bits(int m) { return m <= 1 ? 0 : 32 - __builtin_clz((unsigned)(m - 1)); }
// rank of every product's row in its C column (binary search of C's sorted
// rows), for the backward view
hipError_t launch_bw_dst(const Prob &p, const int2 *E, const long long *pofs, const int32_t *bcol,
                         const int32_t *cri, uint32_t *dst, int *err, hipStream_t s);

// Backward view, built once per single-problem plan: per stored B entry its
// first product (pofs) and its column's first C entry (cb); per stored A entry
// (column, offset in the column); a row view of B (rowptr over B's rows,
// entries by ascending column) holding (B entry, cb) and the first product.
struct BwView {
    const int2 *E;            // the plan's (A column start, length) per stored B entry
    const uint32_t *dst;      // rank of every product's row in its C column
    long long nnzc;           // stored entries of C
    const long long *pofs;    // [nnz(B)]
    const int32_t *cb;        // [nnz(B)]
    const int2 *aview;        // [nnz(A)]
    const int32_t *rowptr;    // [rows of B + 1]
    const int2 *rv;           // [nnz(B)]
    const long long *rvp;     // [nnz(B)]
};
// writable arrays of the view and its construction temporaries
struct BwBuild {
    long long *pofs;
    int32_t *cb;
    int2 *aview;
    int32_t *rowptr;
    int2 *rv;
    long long *rvp;
    int32_t *fill, *colj, *pos, *bcol, *len;
    long long *scratch;  // scan partials of the row counts (nscratch)
    int nscratch;
    long long *scratch2;  // scan partials of the product counts (nscratch2)
    int nscratch2;
    uint32_t *dst;        // [products] rank of every product's row in its C column
};
hipError_t launch_bw_view(const Prob &p, const int2 *E, const BwBuild &b, BwView &w,
                          hipStream_t s);
// dA (if da) and dB (if db) of one problem through the view; err collects
// ERR_CSC for a destination outside C (an inconsistent plan)
hipError_t launch_backward(const Prob &p, const BwView &w, bool f64, const void *av,
                           const void *bv, const void *gv, void *da, void *db, int *err,
                           hipStream_t s);
// nwords 32-bit words from src to mapped host memory dst, as 8-byte pairs
// (word, seq)
hipError_t launch_publish(const void *src, int nwords, void *dst, uint32_t seq, hipStream_t s);
// exclusive scans of n int32 values (bsum: nbsum partials, in place allowed
// for the int32 output)
hipError_t launch_scan_i32(const int32_t *in, int n, long long *bsum, int nbsum, int32_t *out,
                           hipStream_t s);
hipError_t launch_scan_i64(const int32_t *in, int n, long long *bsum, int nbsum, long long *out,
                           hipStream_t s);

constexpr int kScanBlock = 1024;  // elements per scan block

}  // namespace spg
