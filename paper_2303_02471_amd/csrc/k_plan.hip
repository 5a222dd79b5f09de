// Planning kernels: per-column product count Op_j (Section 3.1), accumulator
// choice (the role of the paper's sort + hybrid switch, Sections 3.1-3.3),
// placement of columns into per-accumulator lists, and the column-pointer scan.
#include "devutil.h"

namespace spg {

// ---------------------------------------------------------------- classify
// One workgroup per tile of at most kTile columns of one problem. The tile's
// stored B entries are contiguous; threads walk them flat (coalesced reads of
// B.rowidx, gathers of A.colptr), and add Z^A_k to the owning column's count.
// Every index read here is checked before it is used as an address.
__global__ __launch_bounds__(kBlock) void k_classify(KArgs a) {
    __shared__ int s_bcp[kTile + 1];
    __shared__ unsigned long long s_op[kTile];
    __shared__ int s_hist[NBINS];
    __shared__ int s_err, s_maxch;
    __shared__ unsigned long long s_tot;

    int pid, j0, j1;
    if (a.nprob == 1) {
        pid = 0;
        j0 = blockIdx.x * kTile;
        j1 = min(a.single.n, j0 + kTile);
    } else {
        int4 tl = a.tiles[blockIdx.x];
        pid = tl.x; j0 = tl.y; j1 = tl.z;
    }
    const Prob d = get_prob(a, pid);
    const int nt = j1 - j0;
    const int tid = threadIdx.x;

    for (int c = tid; c <= nt; c += kBlock) s_bcp[c] = d.bcp[j0 + c];
    for (int c = tid; c < nt; c += kBlock) s_op[c] = 0;
    if (tid < NBINS) s_hist[tid] = 0;
    if (tid == 0) { s_err = 0; s_tot = 0; s_maxch = 0; }
    __syncthreads();

    // column pointers of B: monotone, inside [0, nnz], 0 first, nnz last
    int err = 0;
    for (int c = tid; c < nt; c += kBlock)
        if (s_bcp[c + 1] < s_bcp[c]) err = ERR_CSC;
    if (tid == 0) {
        if (s_bcp[0] < 0 || s_bcp[nt] > d.nnzb) err = ERR_CSC;
        if (j0 == 0 && s_bcp[0] != 0) err = ERR_CSC;
        if (j1 == d.n && s_bcp[nt] != d.nnzb) err = ERR_CSC;
        if (j0 == 0) {  // once per problem: A's first and last column pointer
            if (d.acp[0] != 0 || d.acp[d.k] != d.nnza) err = ERR_CSC;
        }
    }
    if (err) atomicOr(&s_err, err);
    __syncthreads();
    if (s_err) {
        if (tid == 0) atomicOr(&a.hdr->err, s_err);
        return;
    }

    const int pb = s_bcp[0], pe = s_bcp[nt];
    const gmem<const int32_t> *__restrict__ bri = to_gmem(d.bri);
    err = 0;
    // with no A columns every stored B entry is out of range (and A.colptr
    // holds one entry: the pair loads below need two)
    const int pe_ok = d.k > 0 ? pe : pb;
    if (d.k == 0 && pe > pb) err = ERR_CSC;
    for (int p0 = pb; p0 < pe_ok; p0 += 4 * kBlock) {
        // Every load of the pass is issued before any is used: a slot past
        // the tile's end reads its last entry, an index out of range reads
        // A's first column pointers; neither result is used.
        int kk[4], x0[4], x1[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) kk[u] = bri[min(p0 + u * kBlock + tid, pe - 1)];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            // both column pointers in one 8-byte load (4-byte alignment is
            // enough for a global load): kc < k, so kc + 1 <= k stays inside
            const int kc = (kk[u] < 0 || kk[u] >= d.k) ? 0 : kk[u];
            const int2a x = load_pair(d.acp, kc);
            x0[u] = x.x;
            x1[u] = x.y;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int p = p0 + u * kBlock + tid;
            const int k = kk[u];
            const bool in = p < pe;
            const bool ok = k >= 0 && k < d.k && x0[u] >= 0 && x1[u] >= x0[u] && x1[u] <= d.nnza;
            const int s0 = ok ? x0[u] : 0, z = (in && ok) ? x1[u] - x0[u] : 0;
            if (in && !ok) err = ERR_CSC;
            // the A column each stored B entry selects, for the accumulators
            if (in) a.E[d.ebase + p] = make_int2(s0, z);
            if (z > 0) atomicAdd(&s_op[last_le(s_bcp, nt + 1, p)], (unsigned long long)z);
        }
    }
    if (err) atomicOr(&s_err, err);
    __syncthreads();
    if (s_err) {
        if (tid == 0) atomicOr(&a.hdr->err, s_err);
        return;
    }

    const int esc_max = 4 << (a.tune.esc_bins - 1);
    unsigned long long tot = 0;
    int maxch = 0;
    err = 0;
    for (int c = tid; c < nt; c += kBlock) {
        const int g = d.col0 + j0 + c;
        unsigned long long op64 = s_op[c];
        if (op64 > 0x7fffffffull) { err = ERR_OPOVF; op64 = 0x7fffffffull; }
        tot += op64;
        const int op = (int)op64;
        // the sort-merge bins take a column by its products or its stored B
        // entries, whichever is more (a work item holds both)
        const int size = max(op, s_bcp[c + 1] - s_bcp[c]);
        int bin;
        if (op == 0) bin = BIN_EMPTY;
        else if (size <= esc_max) bin = BIN_ESC0 + max(ceil_log2(size), 2) - 2;
        else if (op > a.tune.t_block) bin = BIN_BLK0 + blk_class(op);
        else if (size <= kSortMax) bin = BIN_SORT0 + max(ceil_log2(size), 9) - 9;
        else bin = BIN_WSORT;
        if (op > a.tune.t_split) maxch = max(maxch, ceil_div(s_bcp[c + 1] - s_bcp[c], kChunkB));
        a.op[g] = op;
        a.binw[g] = bin;
        a.gnnz[g] = 0;
        atomicAdd(&s_hist[bin], 1);
    }
    if (err) atomicOr(&s_err, err);
    // tile total of products
    atomicAdd(&s_tot, tot);
    if (maxch) atomicMax(&s_maxch, maxch);
    __syncthreads();
    // the tile's tallies (no device atomics: k_tally combines the tiles)
    if (tid < NBINS) a.th[blockIdx.x * NBINS + tid] = s_hist[tid];
    if (tid == 0) {
        a.ttot[blockIdx.x] = (long long)s_tot;
        a.tmax[blockIdx.x] = s_maxch;
        if (s_err) atomicOr(&a.hdr->err, s_err);
    }
}

// ---------------------------------------------------------------- tally
// Workgroup b < NBINS: exclusive scan of bin b's per-tile counts (in place:
// each tile's first position inside the bin) and the bin's total. Workgroup
// NBINS: the product total and the largest chunk count.
__global__ __launch_bounds__(256) void k_tally(KArgs a) {
    constexpr int T = 256, PT = 8;  // threads, consecutive tiles per thread
    __shared__ int tmp[T / 64 + 1];
    __shared__ unsigned long long s_tot;
    __shared__ int s_max;
    const int tid = threadIdx.x, b = blockIdx.x, nt = a.ntiles;
    if (b < NBINS) {
        int carry = 0;
        for (int t0 = 0; t0 < nt; t0 += T * PT) {
            const int tb = t0 + tid * PT;
            int v[PT], sum = 0;
#pragma unroll
            for (int u = 0; u < PT; ++u) {
                v[u] = tb + u < nt ? a.th[(tb + u) * NBINS + b] : 0;
                sum += v[u];
            }
            int total;
            int run = carry + wg_excl_scan<T>(sum, tmp, total);
#pragma unroll
            for (int u = 0; u < PT; ++u) {
                if (tb + u < nt) a.th[(tb + u) * NBINS + b] = run;
                run += v[u];
            }
            carry += total;
        }
        if (tid == 0) {
            a.hdr->bin_count[b] = carry;
            // a planned launch that does not cover a non-empty bin is redone
            if (a.spec_total >= 0 && carry > 0 && !((a.spec_mask >> b) & 1u))
                atomicOr(&a.hdr->err, ERR_RETRY);
        }
    } else {
        if (tid == 0) {
            s_tot = 0;
            s_max = 0;
        }
        __syncthreads();
        unsigned long long tot = 0;
        int mx = 0;
        for (int t0 = 0; t0 < nt; t0 += T * PT) {
#pragma unroll
            for (int u = 0; u < PT; ++u) {
                const int t = t0 + u * T + tid;
                if (t < nt) {
                    tot += (unsigned long long)a.ttot[t];
                    mx = max(mx, a.tmax[t]);
                }
            }
        }
        atomicAdd(&s_tot, tot);
        atomicMax(&s_max, mx);
        __syncthreads();
        if (tid == 0) {
            a.hdr->total_op = s_tot;
            a.hdr->big_chunks = s_max;
            // a planned launch sized for another product count is redone
            if (a.spec_total >= 0 && s_tot != (unsigned long long)a.spec_total)
                atomicOr(&a.hdr->err, ERR_RETRY);
        }
    }
}

hipError_t launch_tally(const KArgs &a, hipStream_t s) {
    if (a.ntiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tally, dim3(NBINS + 1), dim3(256), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------- place
// Same tiling. Each tile writes its columns to its range of every bin list
// (the tally's per-tile positions) in column order, so the columns that one
// wavefront of an accumulator takes lie close together (their per-column
// data and their output in C share cache lines). The rank of a column inside
// its bin is counted with wavefront ballots per bin, then the counts of the
// waves before it.
__global__ __launch_bounds__(kBlock) void k_place(KArgs a) {
    constexpr int PER = kTile / kBlock, NW = kBlock / 64;
    __shared__ int s_start[NBINS];
    __shared__ int s_cnt[PER * NW][NBINS];  // columns of every bin per (pass, wave), then prefix

    if (__syncthreads_or((__atomic_load_n(&a.hdr->err, __ATOMIC_RELAXED) & (ERR_CSC | ERR_OPOVF)) != 0))
        return;  // every thread takes the same branch
    int pid, j0, j1;
    if (a.nprob == 1) {
        pid = 0;
        j0 = blockIdx.x * kTile;
        j1 = min(a.single.n, j0 + kTile);
    } else {
        int4 tl = a.tiles[blockIdx.x];
        pid = tl.x; j0 = tl.y; j1 = tl.z;
    }
    const int col0 = a.nprob == 1 ? 0 : a.table[pid].col0;
    const int nt = j1 - j0;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    if (tid == 0) {
        int run = 0;
        for (int b = 0; b < NBINS; ++b) {
            s_start[b] = run;
            run += a.hdr->bin_count[b];
        }
    }
    // column c = 64 (NW u + w) + lane: passes and waves in column order; the
    // column's entries and product count load together with its bin
    const int32_t *bcp = a.nprob == 1 ? a.single.bcp : a.table[pid].bcp;
    int rank[PER], binv[PER], opv[PER];
    int2a bse[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int c = 64 * (NW * u + w) + lane;
        const bool in = c < nt;
        binv[u] = in ? a.binw[col0 + j0 + c] : -1;
        bse[u] = in ? load_pair(bcp, j0 + c) : int2a{0, 0};
        opv[u] = in ? a.op[col0 + j0 + c] : 0;
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        rank[u] = 0;
        for (int b = 0; b < NBINS; ++b) {
            const unsigned long long m = ballot(binv[u] == b);
            if (binv[u] == b) rank[u] = popc64(m & mask_lt());
            if (lane == 0) s_cnt[NW * u + w][b] = popc64(m);
        }
    }
    __syncthreads();
    // exclusive prefix over (pass, wave) per bin, from the tile's first
    // position in the bin
    if (tid < NBINS) {
        int run = s_start[tid] + a.th[blockIdx.x * NBINS + tid];
        for (int x = 0; x < PER * NW; ++x) {
            const int v = s_cnt[x][tid];
            s_cnt[x][tid] = run;
            run += v;
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int c = 64 * (NW * u + w) + lane;
        if (c >= nt) continue;
        const int g = col0 + j0 + c;
        a.binlist[s_cnt[NW * u + w][binv[u]] + rank[u]] =
            make_int4(g, bse[u].x, bse[u].y - bse[u].x, opv[u]);
    }
}

// ---------------------------------------------------------------- scans
// Exclusive prefix sums in 64-bit, in two launches: per-block sums, then a
// down-sweep in which every block adds up the sums of the blocks before it
// itself (at most a few thousand values) and scans its kScanBlock elements.
// The product-space down-sweep also marks the tile starts.
__global__ __launch_bounds__(kBlock) void k_scan_reduce(const int32_t *__restrict__ in, int n,
                                                        long long *__restrict__ bsum) {
    __shared__ long long s[kBlock / 64];
    const int base = blockIdx.x * kScanBlock;
    long long v = 0;
#pragma unroll
    for (int u = 0; u < kScanBlock / kBlock; ++u) {
        int i = base + u * kBlock + threadIdx.x;
        if (i < n) v += in[i];
    }
    // wave reduction through 32-bit halves
    for (int d = 32; d >= 1; d >>= 1) {
        int lo = (int)(unsigned)v, hi = (int)(unsigned)((unsigned long long)v >> 32);
        lo = __builtin_amdgcn_ds_bpermute((lane_id() ^ d) << 2, lo);
        hi = __builtin_amdgcn_ds_bpermute((lane_id() ^ d) << 2, hi);
        v += (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
    }
    if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        long long t = 0;
        for (int w = 0; w < kBlock / 64; ++w) t += s[w];
        bsum[blockIdx.x] = t;
    }
}

// Block-level scan of kScanBlock int32 values starting at `base` (zero past
// n). Returns, per thread, the exclusive prefixes of its PER consecutive
// elements (global: including the sums of the earlier blocks) and the total
// of all blocks up to this one.
struct ScanOut {
    static constexpr int PER = kScanBlock / kBlock;
    long long pre[PER];
    long long block_end;  // prefix after this block's last element
};

__device__ __forceinline__ void block_scan_down(const int32_t *__restrict__ in, int n,
                                                const long long *__restrict__ bsum,
                                                long long *s, ScanOut &o) {
    constexpr int PER = ScanOut::PER;
    const int base = blockIdx.x * kScanBlock;
    // sums of the earlier blocks
    long long before = 0;
    for (int b = threadIdx.x; b < (int)blockIdx.x; b += kBlock) before += bsum[b];
    s[threadIdx.x] = before;
    __syncthreads();
    for (int d = kBlock / 2; d >= 1; d >>= 1) {
        if ((int)threadIdx.x < d) s[threadIdx.x] += s[threadIdx.x + d];
        __syncthreads();
    }
    before = s[0];
    __syncthreads();
    for (int u = 0; u < PER; ++u) {
        int i = base + u * kBlock + threadIdx.x;
        s[u * kBlock + threadIdx.x] = i < n ? in[i] : 0;
    }
    __syncthreads();
    long long run = 0;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        o.pre[u] = run;
        run += s[threadIdx.x * PER + u];
    }
    __syncthreads();
    s[threadIdx.x] = run;
    __syncthreads();
    for (int d = 1; d < kBlock; d <<= 1) {
        long long t = threadIdx.x >= d ? s[threadIdx.x - d] : 0;
        __syncthreads();
        s[threadIdx.x] += t;
        __syncthreads();
    }
    const long long off = before + s[threadIdx.x] - run;
#pragma unroll
    for (int u = 0; u < PER; ++u) o.pre[u] += off;
    o.block_end = before + s[kBlock - 1];
}

// C column pointers from the per-column counts. For one problem the int32 column pointers are written
// directly (with an overflow check); for several problems the 64-bit global
// prefix is kept in gcp and k_scan_finish cuts it per problem.
__global__ __launch_bounds__(kBlock) void k_scan_down(KArgs a, long long *__restrict__ gcp,
                                                      const long long *__restrict__ bsum,
                                                      long long *__restrict__ totals) {
    __shared__ long long s[kScanBlock];
    const int n = a.ncols;
    ScanOut o;
    block_scan_down(a.gnnz, n, bsum, s, o);
    int err = 0;
#pragma unroll
    for (int u = 0; u < ScanOut::PER; ++u) {
        const int i = blockIdx.x * kScanBlock + threadIdx.x * ScanOut::PER + u;
        if (i >= n) break;
        const long long v = o.pre[u];
        if (a.nprob == 1) {
            if (v > 0x7fffffffll) err = ERR_NNZOVF;
            a.single.ccp[i] = (int32_t)v;
        } else {
            gcp[i] = v;
        }
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
        const long long total = o.block_end;
        if (a.nprob == 1) {
            if (total > 0x7fffffffll) err = ERR_NNZOVF;
            a.single.ccp[n] = (int32_t)total;
            totals[0] = total;
            // a numeric phase queued behind this scan must not write past the
            // caller's arrays
            if (total > a.out_cap) a.hdr->cap_over = 1;
        } else {
            gcp[n] = total;
        }
    }
    if (err) atomicOr(&a.hdr->err, err);
}

__global__ __launch_bounds__(kBlock) void k_scan_finish(KArgs a, const long long *__restrict__ gcp,
                                                        long long *__restrict__ totals) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < a.ncols) {
        const int pid = find_prob(a, i);
        const Prob &d = a.table[pid];
        long long v = gcp[i] - gcp[d.col0];
        d.ccp[i - d.col0] = (int32_t)v;  // per-problem total checked below
    }
    if (i < a.nprob) {
        const Prob &d = a.table[i];
        long long t = gcp[d.col0 + d.n] - gcp[d.col0];
        if (t > 0x7fffffffll) atomicOr(&a.hdr->err, ERR_NNZOVF);
        d.ccp[d.n] = (int32_t)(t > 0x7fffffffll ? 0x7fffffffll : t);
        totals[i] = t;
    }
}

// First product of every global column (exclusive scan of Op_j), and the
// product-balanced tiles: column g starts the tiles t with
// P(g - 1) < t * kProdTile <= P(g); the tiles after the last column's first
// product are empty.
__global__ __launch_bounds__(kBlock) void k_prod_down(KArgs a, const long long *__restrict__ bsum) {
    __shared__ long long s[kScanBlock];
    if (__syncthreads_or(__atomic_load_n(&a.hdr->err, __ATOMIC_RELAXED) != 0))
        return;  // every thread takes the same branch
    const int n = a.ncols;
    ScanOut o;
    block_scan_down(a.op, n, bsum, s, o);
    // a launch planned from an earlier call's sizes may run before the tally
    // has compared them: products beyond the product space carved for that
    // call stop the expansion here
    if (a.spec_total >= 0 && o.block_end > a.spec_total) {
        if (threadIdx.x == 0) atomicOr(&a.hdr->err, ERR_RETRY);
        return;
    }
#pragma unroll
    for (int u = 0; u < ScanOut::PER; ++u) {
        const int g = blockIdx.x * kScanBlock + threadIdx.x * ScanOut::PER + u;
        if (g >= n) break;
        const long long pg = o.pre[u];
        a.colprod[g] = pg;
        const long long t_hi = pg / kProdTile;
        const long long t_lo = g == 0 ? 0 : (pg - a.op[g - 1]) / kProdTile + 1;
        for (long long t = t_lo; t <= t_hi && t < a.nptiles; ++t) a.tilestart[t] = g;
        if (g == n - 1)
            for (long long t = t_hi + 1; t <= a.nptiles; ++t) a.tilestart[t] = n;
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) a.colprod[n] = o.block_end;
}

// generic exclusive scan of int32 values into int32 (in place allowed)
__global__ __launch_bounds__(kBlock) void k_scan_down_i32(const int32_t *in, int n,
                                                          const long long *__restrict__ bsum,
                                                          int32_t *out) {
    __shared__ long long s[kScanBlock];
    ScanOut o;
    block_scan_down(in, n, bsum, s, o);
    __syncthreads();  // every block element is read before any is written (in place)
#pragma unroll
    for (int u = 0; u < ScanOut::PER; ++u) {
        const int i = blockIdx.x * kScanBlock + threadIdx.x * ScanOut::PER + u;
        if (i < n) out[i] = (int32_t)o.pre[u];
    }
}

__global__ __launch_bounds__(kBlock) void k_scan_down_i64(const int32_t *in, int n,
                                                          const long long *__restrict__ bsum,
                                                          long long *out) {
    __shared__ long long s[kScanBlock];
    ScanOut o;
    block_scan_down(in, n, bsum, s, o);
#pragma unroll
    for (int u = 0; u < ScanOut::PER; ++u) {
        const int i = blockIdx.x * kScanBlock + threadIdx.x * ScanOut::PER + u;
        if (i < n) out[i] = o.pre[u];
    }
}

// ---------------------------------------------------------------- launchers
hipError_t launch_scan_i32(const int32_t *in, int n, long long *bsum, int nbsum, int32_t *out,
                           hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int nblk = ceil_div(n, kScanBlock);
    if (nblk > nbsum) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_scan_reduce, dim3(nblk), dim3(kBlock), 0, s, in, n, bsum);
    hipLaunchKernelGGL(k_scan_down_i32, dim3(nblk), dim3(kBlock), 0, s, in, n,
                       (const long long *)bsum, out);
    return hipGetLastError();
}

hipError_t launch_scan_i64(const int32_t *in, int n, long long *bsum, int nbsum, long long *out,
                           hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int nblk = ceil_div(n, kScanBlock);
    if (nblk > nbsum) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_scan_reduce, dim3(nblk), dim3(kBlock), 0, s, in, n, bsum);
    hipLaunchKernelGGL(k_scan_down_i64, dim3(nblk), dim3(kBlock), 0, s, in, n,
                       (const long long *)bsum, out);
    return hipGetLastError();
}

hipError_t launch_prod_offsets(const KArgs &a, long long *bsum, int nbsum, hipStream_t s) {
    if (a.ncols <= 0) return hipSuccess;
    const int nblk = ceil_div(a.ncols, kScanBlock);
    if (nblk > nbsum) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_scan_reduce, dim3(nblk), dim3(kBlock), 0, s, (const int32_t *)a.op,
                       a.ncols, bsum);
    hipLaunchKernelGGL(k_prod_down, dim3(nblk), dim3(kBlock), 0, s, a, (const long long *)bsum);
    return hipGetLastError();
}

hipError_t launch_classify(const KArgs &a, hipStream_t s) {
    if (a.ntiles == 0) return hipSuccess;
    hipLaunchKernelGGL(k_classify, dim3(a.ntiles), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_place(const KArgs &a, hipStream_t s) {
    if (a.ntiles == 0) return hipSuccess;
    hipLaunchKernelGGL(k_place, dim3(a.ntiles), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_scan(const KArgs &a, long long *gcp, long long *bsum, int nblk,
                       long long *totals, hipStream_t s) {
    if (a.ncols > 0) {
        hipLaunchKernelGGL(k_scan_reduce, dim3(nblk), dim3(kBlock), 0, s,
                           (const int32_t *)a.gnnz, a.ncols, bsum);
        hipLaunchKernelGGL(k_scan_down, dim3(nblk), dim3(kBlock), 0, s, a, gcp,
                           (const long long *)bsum, totals);
    }
    if (a.nprob > 1) {
        int n = a.ncols > a.nprob ? a.ncols : a.nprob;
        hipLaunchKernelGGL(k_scan_finish, dim3(ceil_div(n, kBlock)), dim3(kBlock), 0, s, a,
                           (const long long *)gcp, totals);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------- publish
// Copies the header and the per-problem totals (nwords 32-bit words) to mapped
// host memory, each word beside the call's sequence number in one 8-byte
// store, so the host can read them as soon as the symbolic phase ends while
// later work stays queued behind it. A word is current when its pair carries
// the current number: no fence or cache write-back is needed.
__global__ __launch_bounds__(64) void k_publish(const uint32_t *__restrict__ src, int nwords,
                                                unsigned long long *dst, uint32_t seq) {
    for (int i = threadIdx.x; i < nwords; i += 64)
        __hip_atomic_store(&dst[i], (unsigned long long)src[i] | ((unsigned long long)seq << 32),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

hipError_t launch_publish(const void *src, int nwords, void *dst, uint32_t seq, hipStream_t s) {
    hipLaunchKernelGGL(k_publish, dim3(1), dim3(64), 0, s, (const uint32_t *)src, nwords,
                       (unsigned long long *)dst, seq);
    return hipGetLastError();
}

}  // namespace spg
