// Global ESC with radix sort (Section 4), an alternative accumulator for the
// heavy columns (more than 1024 products; option SPGEMM_RADIX_ESC).
//
// Expand: the heavy columns' products are written to the heavy scratch in
// Algorithm 1's order by the heavy expansion (one row and, in the numeric
// phase, one value A(i,k) B(k,j) per product). Consecutive heavy columns form
// a group once their products reach 10,000 (the group threshold of Section
// 4): a column whose first product lies in [10000 g, 10000 (g + 1)) of the
// heavy scratch belongs to group g.
//
// Sort: one workgroup per group sorts the group's product indices by row and
// then by group-local column with a least-significant-digit radix sort of r
// bits per round (r = 5, or 6 when that takes fewer rounds, as Section 4
// chooses). As in the paper's vector version, each of the T = 256 threads
// (its virtual processors) owns a contiguous slice of the current order and
// 2^r buckets; a round counts every slice's digits, scans the counts in
// (digit, thread) order and scatters every slice in order, so the sort is
// stable and equal (column, row) pairs stay in product order. The indices
// ping-pong between two scratch arrays (global memory).
//
// Compress: each thread counts the heads of the equal-key runs in its slice;
// a run's head adds the run's values in order (reading past its slice when
// the run continues) and writes the entry at its column's place in C.
#include "devutil.h"

namespace spg {

constexpr int kRadixGroup = 10000;  // products that close a group (Section 4)
constexpr int kRadixT = 256;        // threads (virtual processors) per group
constexpr int kRadixMaxCols = 64;   // columns of one group (heavy columns: at most 10)
constexpr int kRadixMaxR = 6;       // largest radix length

__device__ __forceinline__ int bit_len(unsigned x) { return x == 0 ? 0 : 32 - __builtin_clz(x); }

template <typename V, bool FILL>
__global__ __launch_bounds__(kRadixT) void k_esc_radix(KArgs a, int rowbits) {
    constexpr int T = kRadixT;
    __shared__ unsigned hist[(1 << kRadixMaxR) * T];  // digit-major: hist[d T + t]
    __shared__ int s_cs[kRadixMaxCols + 1];  // first product of every column (group-local)
    __shared__ int s_cn[kRadixMaxCols];      // output entries of every column
    __shared__ int s_ch[kRadixMaxCols + 1];  // first output entry (head) of every column
    __shared__ int s_lim[2], scan_tmp[T / 64 + 1];
    if (__syncthreads_or((__atomic_load_n(&a.hdr->err, __ATOMIC_RELAXED) |
                          (FILL ? __atomic_load_n(&a.hdr->cap_over, __ATOMIC_RELAXED) : 0)) != 0))
        return;
    int first = 0;
    for (int b = 0; b < BIN_SORT2; ++b) first += a.hdr->bin_count[b];
    int n = 0;
    for (int b = BIN_SORT2; b <= BIN_WSORT; ++b) n += a.hdr->bin_count[b];
    const long long total = a.hoff[n];
    const int nid = (int)(total / kRadixGroup) + 1;
    const int tid = threadIdx.x;
    int bad = 0, depth = 0;
    for (int gid = blockIdx.x; gid < nid; gid += gridDim.x) {
        // the group's columns: first products in [lo, hi)
        if (tid < 2) {
            const long long x = (long long)(gid + tid) * kRadixGroup;
            int l = 0, h = n;  // first li in [0, n] with hoff[li] >= x
            while (l < h) {
                const int mid = (l + h) >> 1;
                if (a.hoff[mid] < x) l = mid + 1;
                else h = mid;
            }
            s_lim[tid] = l;
        }
        __syncthreads();
        const int l0 = s_lim[0], l1 = s_lim[1], nc = l1 - l0;
        __syncthreads();
        if (nc <= 0) continue;
        if (nc > kRadixMaxCols) {  // cannot happen: heavy columns hold more than 1024 products
            bad = 1;
            break;
        }
        const long long base = a.hoff[l0];
        const int np = (int)(a.hoff[l1] - base);
        for (int c = tid; c <= nc; c += T) {
            s_cs[c] = (int)(a.hoff[l0 + c] - base);
            if (c < nc) s_cn[c] = 0;
        }
        __syncthreads();
        const unsigned *__restrict__ rows = (const unsigned *)a.hrow + base;
        unsigned *P[2] = {a.hperm + base, a.hperm + a.heavy_cap + base};
        const int colbits = bit_len((unsigned)(nc - 1));
        // radix length: 5, or 6 when it takes fewer rounds
        const int r5 = ceil_div(rowbits, 5) + ceil_div(colbits, 5);
        const int r6 = ceil_div(rowbits, 6) + ceil_div(colbits, 6);
        const int r = r6 < r5 ? 6 : 5, nb = 1 << r;
        const int rrounds = ceil_div(rowbits, r), rounds = rrounds + ceil_div(colbits, r);
        // group-local column of product e (last column starting at or before e)
        auto col_of = [&](unsigned e) {
            int l = 0, h = nc;
            while (h - l > 1) {
                const int mid = (l + h) >> 1;
                if ((unsigned)s_cs[mid] <= e) l = mid;
                else h = mid;
            }
            return l;
        };
        const int lo_t = (int)((long long)np * tid / T), hi_t = (int)((long long)np * (tid + 1) / T);
        int src = -1;  // current order: identity (product order) or P[src]
        for (int rd = 0; rd < rounds; ++rd) {
            const bool rowf = rd < rrounds;
            const int shift = (rowf ? rd : rd - rrounds) * r;
            auto digit = [&](unsigned e) {
                const unsigned v = rowf ? rows[e] : (unsigned)col_of(e);
                return (int)((v >> shift) & (unsigned)(nb - 1));
            };
            for (int d = 0; d < nb; ++d) hist[d * T + tid] = 0;
            for (int i = lo_t; i < hi_t; ++i) {
                const unsigned e = src < 0 ? (unsigned)i : P[src][i];
                ++hist[digit(e) * T + tid];
            }
            __syncthreads();
            // bucket starts: exclusive scan in (digit, thread) order
            unsigned run = 0;
            for (int k = 0; k < nb; ++k) run += hist[tid * nb + k];
            int tot;
            unsigned acc = (unsigned)block_excl_scan((int)run, scan_tmp, tot);
            for (int k = 0; k < nb; ++k) {
                const unsigned v = hist[tid * nb + k];
                hist[tid * nb + k] = acc;
                acc += v;
            }
            __syncthreads();
            const int dst = src < 0 ? 0 : 1 - src;
            for (int i = lo_t; i < hi_t; ++i) {
                const unsigned e = src < 0 ? (unsigned)i : P[src][i];
                const int d = digit(e);
                P[dst][hist[d * T + tid]++] = e;
            }
            __syncthreads();
            src = dst;
        }
        auto at = [&](int i) { return src < 0 ? (unsigned)i : P[src][i]; };
        auto same = [&](unsigned e, unsigned f) {
            return rows[e] == rows[f] && col_of(e) == col_of(f);
        };
        // run heads of the slice, per column
        int heads = 0;
        for (int i = lo_t; i < hi_t; ++i) {
            const unsigned e = at(i);
            if (i == 0 || !same(at(i - 1), e)) {
                ++heads;
                atomicAdd(&s_cn[col_of(e)], 1);
            }
        }
        int htot;
        const int hbase = block_excl_scan(heads, scan_tmp, htot);
        if (tid == 0) {
            int run = 0;
            for (int c = 0; c < nc; ++c) {
                s_ch[c] = run;
                run += s_cn[c];
            }
            s_ch[nc] = run;
        }
        __syncthreads();
        // columns: counts (symbolic) or positions in C (numeric)
        bool gbad = false;
        for (int c = tid; c < nc; c += T) {
            const int g = a.binlist[first + l0 + c].x;
            if (!FILL || a.spec_fill) a.gnnz[g] = s_cn[c];
            if (FILL) {
                const Prob d = get_prob(a, find_prob(a, g));
                const int j = g - d.col0;
                if (d.ccp[j + 1] - d.ccp[j] != s_cn[c]) gbad = true;  // other inputs
            }
        }
        if (__syncthreads_or(gbad)) {
            bad = 1;
            continue;
        }
        // every head adds its run in order; run lengths give the statistics
        int h = hbase;
        for (int i = lo_t; i < hi_t; ++i) {
            const unsigned e = at(i);
            if (i != 0 && same(at(i - 1), e)) continue;
            const int c = col_of(e);
            int len = 1;
            V accv = V(0);
            if (FILL) accv = V(0) + ((const V *)a.hval)[base + e];
            for (int q = i + 1; q < np; ++q) {
                const unsigned f = at(q);
                if (!same(e, f)) break;
                if (FILL) accv = accv + ((const V *)a.hval)[base + f];
                ++len;
            }
            depth = max(depth, len - 1);
            if (FILL) {
                const int g = a.binlist[first + l0 + c].x;
                const Prob d = get_prob(a, find_prob(a, g));
                const int o = d.ccp[g - d.col0] + (h - s_ch[c]);
                d.cri[o] = (int32_t)rows[e];
                ((V *)d.cv)[o] = accv;
            }
            ++h;
        }
        __syncthreads();
    }
    if ((!FILL || a.spec_fill) && depth > 0) atomicMax(&a.hdr->later_maxk, depth);
    if (bad && tid == 0) atomicOr(&a.hdr->err, FILL && a.spec_fill ? ERR_RETRY : ERR_GROUP);
}

hipError_t launch_esc_radix(const KArgs &a, long long heavy_products, int rowbits, bool fill,
                            bool f64, hipStream_t s) {
    const long long ids = heavy_products / kRadixGroup + 1;
    const dim3 g((unsigned)(ids < 16384 ? ids : 16384)), t(kRadixT);
    if (!fill) hipLaunchKernelGGL((k_esc_radix<float, false>), g, t, 0, s, a, rowbits);
    else if (f64) hipLaunchKernelGGL((k_esc_radix<double, true>), g, t, 0, s, a, rowbits);
    else hipLaunchKernelGGL((k_esc_radix<float, true>), g, t, 0, s, a, rowbits);
    return hipGetLastError();
}

}  // namespace spg
