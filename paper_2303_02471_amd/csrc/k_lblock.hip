// Lane-per-column accumulators fed by the paper's sorting and Blocking
// Algorithm (Section 3.1), for the columns of at most t products (option
// SPGEMM_LANE_BLOCKED; t = t_lane, rounded up to a power of two, <= 64):
//
//   Sorting   the columns by decreasing Op_j (a counting sort over the Op
//             values: the order among equal Op_j is free, as in the paper
//             only the sequence of columns changes, never B);
//   Blocking  from position j: b_min columns, extended while the next
//             column's Op equals the block's first (largest) Op, up to b_max
//             columns or the end (so a block mixes loads only when fewer than
//             b_min columns share one);
//   Blocks    one wavefront per block, one column per lane (the vector
//             element of Algorithm 3), every lane taking one product of its
//             column per step in Algorithm 1's order: B entries in stored
//             order (vIndices_B up to vEnd_B), the A column's entries in
//             stored order (vCounter_A), finished lanes masked.
//
// Accumulators, per lane:
//   HASH   (Section 3.2) a private open-addressing table of H = 2^k slots,
//          2^(k-1) <= max Op_j of the block < 2^k (the table size adapts to
//          every block), h(i) = (i c) mod H with Knuth's multiplicative c,
//          linear probing; keys in LDS, values in global memory (one slab
//          of 128 x 64 slots per wavefront of the launch);
//   SPARS  (Algorithm 3) a private dense accumulator over all m rows: values
//          in global memory (one m x 64 slab per wavefront of the launch),
//          flags as one 64-bit LDS word per row (bit = lane) (m <= 4096).
// Both keep each lane's touched slots or rows in order of first use.
// The first product of a row stores 0 + t and later ones add in order, so
// every value is Algorithm 1's. Each lane then writes its rows in ascending
// order (rank by counting smaller rows) at its column's place in C, or (the
// symbolic phase) its count of distinct rows.
#include "devutil.h"

namespace spg {

constexpr int kLbMaxH = 2 * kLbMaxT;  // largest HASH table (max Op_j = 64 gives 128)

// Stable ranks of a wavefront's active lanes by key: every active lane gets
// the number of active lanes below it with its key; the lowest lane of each
// key (its leader) also gets the key's count. One pass per distinct key.
__device__ __forceinline__ void rank_by_key(int key, bool act, int lane, int &rank, int &cnt,
                                            bool &leader) {
    unsigned long long rem = ballot(act);
    rank = 0;
    cnt = 0;
    leader = false;
    while (rem) {
        const int src = __builtin_ctzll(rem);
        const int k = __builtin_amdgcn_readlane(key, src);
        const bool mine = act && key == k;
        const unsigned long long m = ballot(mine);
        if (mine) {
            rank = popc64(m & mask_lt());
            cnt = popc64(m);
            leader = lane == src;
        }
        rem &= ~m;
    }
}

// Counting sort by decreasing Op: histogram of the lane columns' products.
// Lanes of one value add once per wavefront into LDS, the workgroup once per
// value into the global histogram (columns of one Op would otherwise all
// meet on one address).
__global__ __launch_bounds__(kBlock) void k_lb_hist(KArgs a, LbArgs lb) {
    __shared__ int s_h[kLbMaxT + 1];
    if (__syncthreads_or(__atomic_load_n(&a.hdr->err, __ATOMIC_RELAXED) != 0)) return;
    int start = 0, n = 0;
    for (int b = 0; b < BIN_ESC0; ++b) start += a.hdr->bin_count[b];
    for (int s = 0; s < lb.nsub; ++s) n += a.hdr->bin_count[BIN_ESC0 + s];
    const int tid = threadIdx.x, lane = tid & 63;
    for (int v = tid; v <= kLbMaxT; v += kBlock) s_h[v] = 0;
    __syncthreads();
    bool badop = false;
    for (int i0 = blockIdx.x * kBlock; i0 < n; i0 += gridDim.x * kBlock) {
        const int i = i0 + tid;
        int op = 0;
        if (i < n) {
            op = a.binlist[start + i].w;
            if (op < 1 || op > lb.t) {  // cannot happen
                badop = true;
                op = 0;
            }
        }
        int rk, c;
        bool lead;
        rank_by_key(op, op > 0, lane, rk, c, lead);
        if (lead) atomicAdd(&s_h[op], c);
    }
    __syncthreads();
    for (int v = 1 + tid; v <= lb.t; v += kBlock)
        if (s_h[v]) atomicAdd(&lb.hist[v], s_h[v]);
    if (badop) atomicOr(&a.hdr->err, ERR_GROUP);
}

// Positions of every Op value in the sorted order, then the blocks. One
// thread walks the (at most t) runs of equal Op: a run with at least b_min
// columns left gives blocks of b_max and one of the remainder (if it has
// b_min columns or more); a remainder below b_min opens a block of b_min
// columns reaching into the next runs. Descriptors (first position, blocks,
// block size, first block index); the block total goes to lb.counts[0].
__global__ __launch_bounds__(64) void k_lb_plan(KArgs a, LbArgs lb) {
    if (threadIdx.x != 0) return;
    int n = 0;
    for (int v = lb.t; v >= 1; --v) {
        lb.pos[v] = n;
        n += lb.hist[v];
    }
    if (__atomic_load_n(&a.hdr->err, __ATOMIC_RELAXED)) {
        for (int v = 1; v <= lb.t; ++v) lb.hist[v] = 0;  // zero for the next call
        lb.counts[0] = 0;
        lb.counts[1] = 0;
        return;
    }
    int nd = 0, nblk = 0, j = 0;
    auto emit = [&](int p, int cnt, int size) {
        if (nd < kLbMaxDesc) lb.desc[nd] = make_int4(p, cnt, size, nblk);
        ++nd;
        nblk += cnt;
    };
    // walk: v = Op value at position j, rem = columns of that value from j on
    int v = lb.t;
    while (j < n) {
        while (v >= 1 && lb.pos[v] + lb.hist[v] <= j) --v;  // run holding position j
        const int rem = lb.pos[v] + lb.hist[v] - j;
        if (rem >= lb.b_min) {
            const int q = rem / lb.b_max, r = rem - q * lb.b_max;
            if (q > 0) emit(j, q, lb.b_max);
            j += q * lb.b_max;
            if (r >= lb.b_min) {
                emit(j, 1, r);
                j += r;
            }
            // a remainder below b_min starts the next iteration's spanning block
        } else {
            const int size = min(lb.b_min, n - j);
            emit(j, 1, size);
            j += size;
        }
    }
    if (nd > kLbMaxDesc) atomicOr(&a.hdr->err, ERR_GROUP);  // cannot happen: <= 3 per run
    for (int u = 1; u <= lb.t; ++u) lb.hist[u] = 0;  // zero for the next call
    lb.counts[0] = nblk;
    lb.counts[1] = nd;
}

// Columns into the sorted order (within one Op value in any order): per
// chunk of the workgroup, every Op value reserves its range with one global
// add, every column takes its place by its rank in the chunk.
__global__ __launch_bounds__(kBlock) void k_lb_scatter(KArgs a, LbArgs lb) {
    __shared__ int s_c[kLbMaxT + 1], s_b[kLbMaxT + 1];
    if (__syncthreads_or(__atomic_load_n(&a.hdr->err, __ATOMIC_RELAXED) != 0)) return;
    int start = 0, n = 0;
    for (int b = 0; b < BIN_ESC0; ++b) start += a.hdr->bin_count[b];
    for (int s = 0; s < lb.nsub; ++s) n += a.hdr->bin_count[BIN_ESC0 + s];
    const int tid = threadIdx.x, lane = tid & 63;
    bool over = false;
    for (int i0 = blockIdx.x * kBlock; i0 < n; i0 += gridDim.x * kBlock) {
        for (int v = tid; v <= kLbMaxT; v += kBlock) s_c[v] = 0;
        __syncthreads();
        const int i = i0 + tid;
        int4 ent = make_int4(0, 0, 0, 0);
        if (i < n) ent = a.binlist[start + i];
        const int op = (i < n && ent.w >= 1 && ent.w <= lb.t) ? ent.w : 0;  // else flagged
        int rk, c;
        bool lead;
        rank_by_key(op, op > 0, lane, rk, c, lead);
        // the wavefront's range inside the chunk's count of its value,
        // taken by the key's leader and handed to the key's lanes
        int local = 0, wbase = 0;
        if (lead) wbase = atomicAdd(&s_c[op], c);
        {
            unsigned long long rem = ballot(op > 0);
            while (rem) {
                const int src = __builtin_ctzll(rem);
                const int k = __builtin_amdgcn_readlane(op, src);
                const int b = __builtin_amdgcn_readlane(wbase, src);
                const unsigned long long m = ballot(op > 0 && op == k);
                if (op > 0 && op == k) local = b + rk;
                rem &= ~m;
            }
        }
        __syncthreads();
        for (int v = 1 + tid; v <= lb.t; v += kBlock)
            if (s_c[v]) s_b[v] = atomicAdd(&lb.pos[v], s_c[v]);
        __syncthreads();
        if (op > 0) {
            const int at = s_b[op] + local;
            if (at < lb.ncap) lb.sorted[at] = ent;
            else over = true;  // cannot happen
        }
        __syncthreads();
    }
    if (over) atomicOr(&a.hdr->err, ERR_GROUP);
}

// HASH tables (slot h of lane l at h * 64 + l) or SPARS flags and row lists
template <typename V, bool SPARS>
struct LbSmem;
template <typename V>
struct LbSmem<V, false> {
    int key[kLbMaxH * 64];
    uint8_t used[kLbMaxT * 64];  // x-th slot of lane l taken, at x * 64 + l
};
template <typename V>
struct LbSmem<V, true> {
    unsigned long long flag[kSparsMaxRows];
    int idx[kLbMaxT * 64];  // x-th row of lane l touched, at x * 64 + l
};

template <typename V, bool SPARS, bool FILL>
__global__ __launch_bounds__(64) void k_lane_blocked(KArgs a, LbArgs lb) {
    __shared__ LbSmem<V, SPARS> L;
    if (__atomic_load_n(&a.hdr->err, __ATOMIC_RELAXED) |
        (FILL ? __atomic_load_n(&a.hdr->cap_over, __ATOMIC_RELAXED) : 0))
        return;
    const int lane = threadIdx.x;
    const int nblk = lb.counts[0], nd = min(lb.counts[1], kLbMaxDesc);
    // the wavefront's value slab: slot or row x of lane l at x * 64 + l
    V *slab = FILL ? (V *)lb.dense + (size_t)blockIdx.x * (SPARS ? lb.mslab : kLbMaxH) * 64
                   : nullptr;
    if constexpr (SPARS) {
        for (int r = lane; r < kSparsMaxRows; r += 64) L.flag[r] = 0;
        __syncthreads();
    }
    int bad = 0, badrow = 0;
    for (int bi = blockIdx.x; bi < nblk; bi += gridDim.x) {
        // the block's descriptor: last with first block index <= bi
        int lo = 0, hi = nd;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (lb.desc[mid].w <= bi) lo = mid;
            else hi = mid;
        }
        const int4 ds = lb.desc[lo];
        const int bstart = ds.x + (bi - ds.w) * ds.z, bsize = ds.z;
        if (bstart < 0 || bsize < 1 || bsize > 64 || bstart + bsize > lb.ncap) {  // cannot happen
            bad = 1;
            break;
        }
        const bool act0 = lane < bsize;
        int4 ent = make_int4(0, 0, 0, 0);
        if (act0) ent = lb.sorted[bstart + lane];
        const int g = ent.x;
        Prob d{};
        if (act0) d = get_prob(a, find_prob(a, g));
        // table size of the block: its first column has the largest Op
        const int maxop = __builtin_amdgcn_readfirstlane(ent.w);
        int H = 1;
        while (H <= maxop) H <<= 1;
        const int lg = 31 - __builtin_clz((unsigned)H);
        if constexpr (!SPARS)
            for (int h = 0; h < H; ++h) L.key[h * 64 + lane] = -1;
        if (SPARS && act0 && d.m > lb.mslab) bad = 1;  // cannot happen: checked on the host
        // Algorithm 3: vIndices_B, vEnd_B, vCounter_A per lane
        const int2 *__restrict__ Ep = a.E + d.ebase;
        int p = ent.y, pend = ent.y + ent.z, ca = 0, as = 0, z = 0, cnt = 0;
        V bval = V(0);
        bool act = act0 && p < pend && !(SPARS && d.m > lb.mslab);
        while (__builtin_amdgcn_ballot_w64(act)) {
            if (act) {
                if (ca == 0) {
                    const int2 e = Ep[p];
                    as = e.x;
                    z = e.y;
                    if (FILL) bval = ((const V *)d.bv)[p];
                }
                if (z == 0) {
                    ++p;
                    act = p < pend;
                    continue;
                }
                const int i = d.ari[as + ca];
                V t = V(0);
                if (FILL) t = ((const V *)d.av)[as + ca] * bval;
                if (i < 0 || i >= d.m) {
                    badrow = 1;
                } else if constexpr (!SPARS) {
                    int h = (int)(((unsigned)i * 2654435761u) >> (32 - lg));
                    while (L.key[h * 64 + lane] != -1 && L.key[h * 64 + lane] != i) h = (h + 1) & (H - 1);
                    if (L.key[h * 64 + lane] == -1) {
                        L.key[h * 64 + lane] = i;
                        if (FILL) slab[h * 64 + lane] = V(0) + t;
                        L.used[cnt * 64 + lane] = (uint8_t)h;
                        ++cnt;
                    } else if (FILL) {
                        slab[h * 64 + lane] = slab[h * 64 + lane] + t;
                    }
                } else {
                    const unsigned long long bit = 1ull << lane;
                    if (!(L.flag[i] & bit)) {
                        atomicOr(&L.flag[i], bit);
                        if (FILL) slab[(size_t)i * 64 + lane] = V(0) + t;
                        L.idx[cnt * 64 + lane] = i;
                        ++cnt;
                    } else if (FILL) {
                        slab[(size_t)i * 64 + lane] = slab[(size_t)i * 64 + lane] + t;
                    }
                }
                if (++ca == z) {
                    ca = 0;
                    ++p;
                }
                act = p < pend;
            }
        }
        // outputs: rows ascending (rank = count of smaller rows)
        if (act0) {
            if (!FILL || a.spec_fill) a.gnnz[g] = cnt;
            if (FILL) {
                const int j = g - d.col0;
                const int c0 = d.ccp[j], clen = d.ccp[j + 1] - c0;
                if (clen != cnt) {
                    bad = 1;
                } else if constexpr (!SPARS) {
                    for (int x = 0; x < cnt; ++x) {
                        const int h = L.used[x * 64 + lane], r = L.key[h * 64 + lane];
                        int rk = 0;
                        for (int y = 0; y < cnt; ++y)
                            rk += L.key[L.used[y * 64 + lane] * 64 + lane] < r ? 1 : 0;
                        d.cri[c0 + rk] = r;
                        ((V *)d.cv)[c0 + rk] = slab[h * 64 + lane];
                    }
                } else {
                    for (int x = 0; x < cnt; ++x) {
                        const int r = L.idx[x * 64 + lane];
                        int rk = 0;
                        for (int y = 0; y < cnt; ++y) rk += L.idx[y * 64 + lane] < r ? 1 : 0;
                        d.cri[c0 + rk] = r;
                        ((V *)d.cv)[c0 + rk] = slab[(size_t)r * 64 + lane];
                    }
                }
            }
            if constexpr (SPARS)  // clear the lane's flags for the next block
                for (int x = 0; x < cnt; ++x) atomicAnd(&L.flag[L.idx[x * 64 + lane]], ~(1ull << lane));
        }
        __syncthreads();
    }
    if (__builtin_amdgcn_ballot_w64(bad != 0) && lane == 0)
        atomicOr(&a.hdr->err, FILL && a.spec_fill ? ERR_RETRY : ERR_GROUP);
    if (__builtin_amdgcn_ballot_w64(badrow != 0) && lane == 0) atomicOr(&a.hdr->err, ERR_CSC);
}

hipError_t launch_lane_blocked(const KArgs &a, const LbArgs &lb, int ncols_hint, int grid_cap,
                               bool spars, bool fill, bool f64, hipStream_t s) {
    const int g1 = ceil_div(std::max(ncols_hint, 1), kBlock);
    const dim3 gl(g1 < 1024 ? g1 : 1024), tb(kBlock);
    hipLaunchKernelGGL(k_lb_hist, gl, tb, 0, s, a, lb);
    hipLaunchKernelGGL(k_lb_plan, dim3(1), dim3(64), 0, s, a, lb);
    hipLaunchKernelGGL(k_lb_scatter, gl, tb, 0, s, a, lb);
    int blocks = ceil_div(std::max(ncols_hint, 1), std::max(lb.b_min, 1)) + 1;
    if (blocks > grid_cap) blocks = grid_cap;
    const dim3 g(blocks), t(64);
    if (!fill) {
        if (spars) hipLaunchKernelGGL((k_lane_blocked<float, true, false>), g, t, 0, s, a, lb);
        else hipLaunchKernelGGL((k_lane_blocked<float, false, false>), g, t, 0, s, a, lb);
    } else if (f64) {
        if (spars) hipLaunchKernelGGL((k_lane_blocked<double, true, true>), g, t, 0, s, a, lb);
        else hipLaunchKernelGGL((k_lane_blocked<double, false, true>), g, t, 0, s, a, lb);
    } else {
        if (spars) hipLaunchKernelGGL((k_lane_blocked<float, true, true>), g, t, 0, s, a, lb);
        else hipLaunchKernelGGL((k_lane_blocked<float, false, true>), g, t, 0, s, a, lb);
    }
    return hipGetLastError();
}

}  // namespace spg
