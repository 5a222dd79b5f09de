// Product expansion and the numeric phase.
//
// Product-balanced tiles: tile t holds the columns whose first product lies in
// [t * kProdTile, (t + 1) * kProdTile) of the product space, so every tile has
// about kProdTile products (plus the tail of its last column).
//
// Expansion: one workgroup per kExpandTiles consecutive tiles walks their
// stored B entries in storage order (they are contiguous) and writes the row
// of every product -- the rows of the A column each entry selects, in storage
// order -- to the product space. The symbolic accumulators stream these rows.
//
// Numeric: the symbolic phase left, per product, its row (the expansion) and
// a destination: the rank of its output row inside its column, or for a
// product that is not the first of its output entry a place in the list of
// such "later" products with its occurrence index k. The numeric kernels form
// every product A(i,k) * B(k,j) from the values of the selected A columns,
// read both arrays in product order and write
// the first product of each entry as 0 + product straight to its output
// position; later products are staged, and layer kernels add those of
// occurrence index 1, 2, ... in that order, so every output entry is summed in
// Algorithm 1's order and rounding, bit for bit. Columns of at most t_split
// products go by product-balanced tiles, larger ones by chunks of kChunkB
// stored B entries (one workgroup each), so no workgroup holds a whole large
// column.
#include "devutil.h"

namespace spg {

// Calls f(pid, d, j0, j1) for the problem segments of tile columns [g0, g1).
template <typename F>
__device__ __forceinline__ void for_each_segment(const KArgs &a, int g0, int g1, F &&f) {
    int g = g0;
    while (g < g1) {
        const int pid = find_prob(a, g);
        const Prob d = get_prob(a, pid);
        const int gend = min(g1, d.col0 + d.n);
        f(pid, d, g - d.col0, gend - d.col0);
        g = gend;
    }
}

// ---------------------------------------------------------------- expansion
struct ExpSmem {
    int s_acp[kBlock];   // A column start of each stored B entry of the B window
    int s_eoff[kBlock];  // first product of each stored B entry of the B window
    int scan_tmp[kBlock / 64 + 1];
};

// product tiles per expansion workgroup (1, 2, 8 and 16 measured slower)
constexpr int kExpandTiles = 4;

__global__ __launch_bounds__(kBlock) void k_expand(KArgs a) {
    constexpr int PER = 4;
    __shared__ ExpSmem S;
    if (__syncthreads_or(__atomic_load_n(&a.hdr->err, __ATOMIC_RELAXED) != 0))
        return;  // every thread takes the same branch
    const int tid = threadIdx.x;
    const int t0 = (int)blockIdx.x * kExpandTiles;
    const int g0 = a.tilestart[t0], g1 = a.tilestart[min(t0 + kExpandTiles, a.nptiles)];
    int *__restrict__ prow = a.prow;
    int bad = 0;
    for_each_segment(a, g0, g1, [&](int, const Prob &d, int j0, int j1) {
        long long base = a.colprod[d.col0 + j0];
        const gmem<const int32_t> *bcp = to_gmem(d.bcp);
        const int pb = bcp[j0], pe = bcp[j1];  // checked by the classification
        const int2 *__restrict__ Ep = a.E + d.ebase;
        const gmem<const int32_t> *__restrict__ ari = to_gmem(d.ari);
        for (int bw = pb; bw < pe; bw += kBlock) {
            const int t = bw + tid;
            int z = 0, acp = 0;
            if (t < pe) {
                const int2 ez = Ep[t];
                acp = ez.x;
                z = ez.y;
            }
            int Ew;
            const int ex = block_excl_scan(z, S.scan_tmp, Ew);
            S.s_acp[tid] = acp;
            S.s_eoff[tid] = ex;
            __syncthreads();
            const int nbw = min(kBlock, pe - bw);
            for (int e0 = 0; e0 < Ew; e0 += PER * kBlock) {
                int r[PER];
#pragma unroll
                for (int u = 0; u < PER; ++u) {
                    const int e = e0 + u * kBlock + tid;
                    r[u] = 0;
                    if (e < Ew) {
                        const int tt = last_le(S.s_eoff, nbw, e);
                        r[u] = ari[S.s_acp[tt] + e - S.s_eoff[tt]];
                    }
                }
#pragma unroll
                for (int u = 0; u < PER; ++u) {
                    const int e = e0 + u * kBlock + tid;
                    if (e >= Ew) continue;
                    int row = r[u];
                    if (row < 0 || row >= d.m) {
                        bad |= ERR_CSC;
                        row = 0;
                    }
                    // the A column lengths (E) and the product offsets (from
                    // Op_j) agree unless the inputs changed under the plan:
                    // never write beyond the product space
                    if (base + e >= a.prod_cap) {
                        bad |= ERR_GROUP;
                        continue;
                    }
                    prow[base + e] = row;
                }
            }
            base += Ew;
            __syncthreads();
        }
    });
    if (bad) atomicOr(&a.hdr->err, bad);
}

hipError_t launch_expand(const KArgs &a, hipStream_t s) {
    if (a.nptiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_expand, dim3(ceil_div(a.nptiles, kExpandTiles)), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------- numeric
// Forms the products of `nbw` stored B entries (window arrays in LDS: A
// column start, first product of the entry in the window's product numbering,
// window column, B value) and writes each product through its destination:
// the first product of an entry as first(c, rank, row, 0 + product), a later
// product into the staging of the later list. `pos(tt, e)` gives the
// product-space index of product e (window numbering) of entry tt,
// `cinfo(c, c0, clen, lb)` the column's output start and length and the start
// of its later products in the compact list.
template <typename V, int PER, typename Pos, typename Cinfo, typename First>
__device__ __forceinline__ void numeric_window(const KArgs &a, int pid, const Prob &d,
                                               const int *s_acp, const int *s_eoff,
                                               const int *s_col, const V *s_bv, int nbw, int Ew,
                                               Pos &&pos, Cinfo &&cinfo, First &&first,
                                               int &bad) {
    const gmem<const V> *__restrict__ av = to_gmem((const V *)d.av);
    V *__restrict__ lv = (V *)a.lv;
    const int tid = threadIdx.x;
    for (int e0 = 0; e0 < Ew; e0 += PER * kBlock) {
        V x[PER], y[PER];
        int row[PER], c[PER];
        uint32_t dc[PER];
        long long pp[PER];
        // All of the thread's loads are issued, without branches, before any
        // is used, so its gathers of A's values are in flight together. A
        // slot past the window's end repeats the window's last product and
        // writes nothing.
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int e = e0 + u * kBlock + tid;
            const int ee = min(e, Ew - 1);
            const int tt = last_le(s_eoff, nbw, ee);
            const int q = s_acp[tt] + ee - s_eoff[tt];
            c[u] = e < Ew ? s_col[tt] : -1;
            pp[u] = pos(tt, ee);
            // a product beyond the product space (inputs changed under the
            // plan) is read at its last position and never written
            if (pp[u] >= a.prod_cap) {
                pp[u] = a.prod_cap - 1;
                if (c[u] >= 0) bad = 1;
                c[u] = -1;
            }
            y[u] = s_bv[tt];
            x[u] = av[q];
            row[u] = a.prow[pp[u]];  // the expansion's row, read in product order
            dc[u] = a.dst[pp[u]];
        }
#pragma unroll
        for (int u = 0; u < PER; ++u) x[u] = x[u] * y[u];
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            if (c[u] < 0) continue;
            const V vu = x[u];
            int c0, clen;
            long long lb;
            cinfo(c[u], c0, clen, lb);
            const int o = (int)(dc[u] & ~kDstLater);
            if (o >= clen) { bad = 1; continue; }
            if (!(dc[u] & kDstLater)) {
                first(c[u], o, row[u], V(0) + vu);
            } else {
                const long long li = lb + a.lr[pp[u]];
                if (li < 0 || li >= a.later_n) { bad = 1; continue; }
                a.lo[li] = c0 + o;
                a.lpid[li] = pid;
                a.lkc[li] = a.lk[pp[u]];
                lv[li] = vu;
            }
        }
    }
}

constexpr int kColWin = 256;  // columns per window of a tile
constexpr int kNumPer = 2;     // products per thread per pass, product-balanced tiles
constexpr int kNumPerBig = 8;  // products per thread per pass, chunks of large columns

template <typename V>
struct NumSmem {
    int s_bcp[kColWin + 1];     // B column pointers of the column window
    int s_c0[kColWin + 1];      // C column pointers of the column window
    int s_ceff[kColWin + 1];    // first product of each column among the window's tile columns
    long long s_pcol[kColWin];  // first product of each column in the product space
    int s_ok[kColWin];          // column done by the tile (at most t_split products)
    long long s_lb[kColWin];    // start of each column's later products in the compact list
    int s_acp[kBlock];          // A column start of each stored B entry of the B window
    int s_eoff[kBlock];         // first product of each stored B entry of the B window
    int s_col[kBlock];          // window column of each stored B entry of the B window
    V s_bv[kBlock];             // B value of each stored B entry of the B window
    int scan_tmp[kBlock / 64 + 1];
};

// One workgroup per product-balanced tile; columns with more than t_split
// products are left to the chunk workgroups (their products count zero here).
template <typename V>
__device__ __forceinline__ void numeric_tile(const KArgs &a, NumSmem<V> &S, int tile) {
    const int tid = threadIdx.x;
    const int g0 = a.tilestart[tile], g1 = a.tilestart[tile + 1];
    if (g0 >= g1) return;
    int bad = 0;
    for_each_segment(a, g0, g1, [&](int pid, const Prob &d, int js, int je) {
        const int2 *__restrict__ Ep = a.E + d.ebase;
        const gmem<const V> *__restrict__ bv = to_gmem((const V *)d.bv);
        const gmem<const int32_t> *__restrict__ bcp = to_gmem(d.bcp);
        const gmem<const int32_t> *__restrict__ ccp = to_gmem((const int32_t *)d.ccp);
        for (int jw = js; jw < je; jw += kColWin) {
            const int nc = min(kColWin, je - jw);
            const int gw = d.col0 + jw;
            int eff = 0;
            for (int c = tid; c <= nc; c += kBlock) {
                S.s_bcp[c] = bcp[jw + c];
                S.s_c0[c] = ccp[jw + c];
            }
            if (tid < nc) {
                const int op = a.op[gw + tid];
                const int ok = op <= a.tune.t_split;
                S.s_ok[tid] = ok;
                const int c0 = ccp[jw + tid];
                const long long pc = a.colprod[gw + tid];
                S.s_pcol[tid] = pc;
                S.s_lb[tid] = pc - (a.nprob == 1 ? (long long)c0 : a.gcp[gw + tid]);
                eff = ok ? op : 0;
            }
            int tot;
            const int ex = block_excl_scan(eff, S.scan_tmp, tot);
            if (tid < nc) S.s_ceff[tid] = ex;
            if (tid == 0) S.s_ceff[nc] = tot;
            __syncthreads();
            gmem<int32_t> *__restrict__ cri = to_gmem(d.cri);
            gmem<V> *__restrict__ cv = to_gmem((V *)d.cv);
            const int pb = S.s_bcp[0], pe = S.s_bcp[nc];
            int base = 0;  // first product of the B window among the tile columns
            int2 nez = make_int2(0, 0);
            V nb = V(0);
            if (pb + tid < pe) {
                nez = Ep[pb + tid];
                nb = bv[pb + tid];
            }
            for (int bw = pb; bw < pe; bw += kBlock) {
                const int t = bw + tid;
                const int2 ez = nez;
                const V b0 = nb;
                if (t + kBlock < pe) {
                    nez = Ep[t + kBlock];
                    nb = bv[t + kBlock];
                }
                int z = 0, col = 0;
                if (t < pe) {
                    col = last_le(S.s_bcp, nc + 1, t);
                    if (S.s_ok[col]) z = ez.y;
                }
                int Ew;
                const int ez0 = block_excl_scan(z, S.scan_tmp, Ew);
                S.s_acp[tid] = ez.x;
                S.s_eoff[tid] = ez0;
                S.s_col[tid] = col;
                S.s_bv[tid] = b0;
                __syncthreads();
                const int nbw = min(kBlock, pe - bw);
                numeric_window<V, kNumPer>(
                    a, pid, d, S.s_acp, S.s_eoff, S.s_col, S.s_bv, nbw, Ew,
                    [&](int tt, int e) {
                        const int c = S.s_col[tt];
                        return S.s_pcol[c] + (base + e - S.s_ceff[c]);
                    },
                    [&](int c, int &c0, int &clen, long long &lb) {
                        c0 = S.s_c0[c];
                        clen = S.s_c0[c + 1] - c0;
                        lb = S.s_lb[c];
                    },
                    [&](int c, int o, int row, V v) {
                        cri[S.s_c0[c] + o] = row;
                        cv[S.s_c0[c] + o] = v;
                    },
                    bad);
                base += Ew;
                __syncthreads();
            }
            // every thread has read this window's bounds (pb, pe) before the
            // next window overwrites them, also when no B entry ran the loop
            __syncthreads();
        }
    });
    if (bad) atomicOr(&a.hdr->err, ERR_GROUP);
}

// ---------------------------------------------------------------- numeric, large columns
template <typename V>
struct BigSmem {
    int s_acp[kBlock];
    int s_eoff[kBlock];
    int s_col[kBlock];
    V s_bv[kBlock];
    int scan_tmp[kBlock / 64 + 1];
    long long s_pre;
};

// One workgroup per chunk of kChunkB stored B entries of a column with more
// than t_split products. Workgroups are dealt to the XCDs round-robin by
// launch order; the numbering below sends every chunk of column c to XCD
// c mod 8, so the column's output lines, written piecewise by its chunks,
// meet in one L2 before they are written back.
constexpr int kXcds = 8;
static_assert(kChunkB % kBlock == 0, "a chunk is a whole number of B windows");

template <typename V>
__device__ __forceinline__ void numeric_chunk(const KArgs &a, BigSmem<V> &S, int first, int n,
                                              int wg) {
    const int tid = threadIdx.x;
    const int ncol8 = ceil_div(n, kXcds);
    const int xcd = wg % kXcds, r = wg / kXcds;
    const int chunk = r / ncol8, col = (r % ncol8) * kXcds + xcd;
    if (col >= n) return;
    const int4 ent = a.binlist[first + col];
    const int g = ent.x, bs = ent.y, nb = ent.z;
    const int op = a.op[g];
    const int b0 = bs + chunk * kChunkB;
    if (op <= a.tune.t_split || b0 >= bs + nb) return;  // tile column, or no such chunk
    const int b1 = min(bs + nb, b0 + kChunkB);
    const int pid = find_prob(a, g);
    const Prob d = get_prob(a, pid);
    const int j = g - d.col0;
    const int2 *__restrict__ Ep = a.E + d.ebase;
    // this chunk's first product: the products of the column's earlier entries
    long long pre = 0;
    for (int x = bs + tid; x < b0; x += kBlock) pre += Ep[x].y;
    if (tid == 0) S.s_pre = 0;
    __syncthreads();
    if (pre) atomicAdd((unsigned long long *)&S.s_pre, (unsigned long long)pre);
    const gmem<const int32_t> *ccp = to_gmem((const int32_t *)d.ccp);
    const int c0 = ccp[j], clen = ccp[j + 1] - c0;
    const long long lb0 = a.colprod[g] - (a.nprob == 1 ? (long long)c0 : a.gcp[g]);
    const gmem<const V> *__restrict__ bv = to_gmem((const V *)d.bv);
    gmem<int32_t> *__restrict__ cri = to_gmem(d.cri);
    gmem<V> *__restrict__ cv = to_gmem((V *)d.cv);
    __syncthreads();
    long long pbase = a.colprod[g] + S.s_pre;
    int bad = 0;
    // the chunk's entries in windows of kBlock, the next window's loads in flight
    int2 nez = make_int2(0, 0);
    V nbv = V(0);
    if (b0 + tid < b1) {
        nez = Ep[b0 + tid];
        nbv = bv[b0 + tid];
    }
    for (int bw = b0; bw < b1; bw += kBlock) {
        const int t = bw + tid;
        const int2 ez = nez;
        const V b = nbv;
        if (t + kBlock < b1) {
            nez = Ep[t + kBlock];
            nbv = bv[t + kBlock];
        }
        int Ew;
        const int ex = block_excl_scan(t < b1 ? ez.y : 0, S.scan_tmp, Ew);
        S.s_acp[tid] = ez.x;
        S.s_eoff[tid] = ex;
        S.s_col[tid] = 0;
        S.s_bv[tid] = b;
        __syncthreads();
        const long long pb = pbase;
        numeric_window<V, kNumPerBig>(
            a, pid, d, S.s_acp, S.s_eoff, S.s_col, S.s_bv, min(kBlock, b1 - bw), Ew,
            [&](int, int e) { return pb + e; },
            [&](int, int &o0, int &ol, long long &lb) {
                o0 = c0;
                ol = clen;
                lb = lb0;
            },
            [&](int, int o, int row, V v) {
                cri[c0 + o] = row;
                cv[c0 + o] = v;
            },
            bad);
        pbase += Ew;
        __syncthreads();
    }
    if (bad) atomicOr(&a.hdr->err, ERR_GROUP);
}

template <typename V>
union NumericSmem {
    NumSmem<V> tile;
    BigSmem<V> chunk;
};

// The numeric launch: workgroups [0, nchunkwg) take the chunks of the
// columns above t_split (listed from bin-list position `first`, `nbig` of
// them; nchunkwg is a multiple of 8 so the XCD numbering holds), the rest one
// product-balanced tile each. One launch lets the two kinds share the chip
// without a fork and join of streams.
template <typename V>
__global__ __launch_bounds__(kBlock) void k_numeric(KArgs a, int first, int nbig, int nchunkwg) {
    __shared__ NumericSmem<V> S;
    if (__syncthreads_or((__atomic_load_n(&a.hdr->err, __ATOMIC_RELAXED) |
                          __atomic_load_n(&a.hdr->cap_over, __ATOMIC_RELAXED)) != 0))
        return;  // every thread takes the same branch
    if ((int)blockIdx.x < nchunkwg) numeric_chunk<V>(a, S.chunk, first, nbig, (int)blockIdx.x);
    else numeric_tile<V>(a, S.tile, (int)blockIdx.x - nchunkwg);
}

// later products of occurrence index k, added to their (already written)
// output entries; every entry has at most one product of each index
template <typename V>
__global__ __launch_bounds__(kBlock) void k_layer(KArgs a, int k, long long n) {
    // a layer queued behind a phase that stood down finds the list of an
    // earlier call: it stands down too, and never writes outside C
    if ((__atomic_load_n(&a.hdr->err, __ATOMIC_RELAXED) |
         __atomic_load_n(&a.hdr->cap_over, __ATOMIC_RELAXED)) != 0)
        return;
    const V *__restrict__ lv = (const V *)a.lv;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (long long)gridDim.x * kBlock) {
        if (a.lkc[i] != k) continue;
        const int pid = a.lpid[i];
        const int o = a.lo[i];
        if (pid < 0 || pid >= a.nprob || o < 0 || (long long)o >= a.out_cap) continue;
        const Prob d = get_prob(a, pid);
        gmem<V> *cv = to_gmem((V *)d.cv);
        cv[o] = cv[o] + lv[i];
    }
}

// All later products in one launch, for later lists in sorted-key order (every
// accumulator but the hash one): the later products of one output entry are
// consecutive there, in occurrence order, so the thread at the head of each
// such run adds the run in order (the same sums as one launch per k).
template <typename V>
__global__ __launch_bounds__(kBlock) void k_later_runs(KArgs a, long long n) {
    if ((__atomic_load_n(&a.hdr->err, __ATOMIC_RELAXED) |
         __atomic_load_n(&a.hdr->cap_over, __ATOMIC_RELAXED)) != 0)
        return;
    const V *__restrict__ lv = (const V *)a.lv;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (long long)gridDim.x * kBlock) {
        const int pid = a.lpid[i];
        const int o = a.lo[i];
        if (i > 0 && a.lo[i - 1] == o && a.lpid[i - 1] == pid) continue;  // inside a run
        if (pid < 0 || pid >= a.nprob || o < 0 || (long long)o >= a.out_cap) continue;
        const Prob d = get_prob(a, pid);
        gmem<V> *cv = to_gmem((V *)d.cv);
        V acc = cv[o];
        for (long long j = i; j < n && a.lo[j] == o && a.lpid[j] == pid; ++j) acc = acc + lv[j];
        cv[o] = acc;
    }
}

hipError_t launch_numeric(const KArgs &a, bool f64, int first, int nbig, int maxchunks,
                          hipStream_t s) {
    const long long nchunk =
        (nbig > 0 && maxchunks > 0) ? (long long)kXcds * ceil_div(nbig, kXcds) * maxchunks : 0;
    const long long nwg = nchunk + (a.nptiles > 0 ? a.nptiles : 0);
    if (nwg <= 0) return hipSuccess;
    if (nwg > 0x7fffffffll) return hipErrorInvalidValue;
    const dim3 grid((unsigned)nwg);
    if (f64)
        hipLaunchKernelGGL((k_numeric<double>), grid, dim3(kBlock), 0, s, a, first, nbig, (int)nchunk);
    else
        hipLaunchKernelGGL((k_numeric<float>), grid, dim3(kBlock), 0, s, a, first, nbig, (int)nchunk);
    return hipGetLastError();
}

hipError_t launch_later_runs(const KArgs &a, bool f64, long long n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const long long want = (n + kBlock - 1) / kBlock;
    const int grid = (int)std::min<long long>(want, 8192);
    if (f64) hipLaunchKernelGGL((k_later_runs<double>), dim3(grid), dim3(kBlock), 0, s, a, n);
    else hipLaunchKernelGGL((k_later_runs<float>), dim3(grid), dim3(kBlock), 0, s, a, n);
    return hipGetLastError();
}

hipError_t launch_layer(const KArgs &a, bool f64, int k, long long n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const long long want = (n + kBlock - 1) / kBlock;
    const int grid = (int)std::min<long long>(want, 8192);
    if (f64) hipLaunchKernelGGL((k_layer<double>), dim3(grid), dim3(kBlock), 0, s, a, k, n);
    else hipLaunchKernelGGL((k_layer<float>), dim3(grid), dim3(kBlock), 0, s, a, k, n);
    return hipGetLastError();
}

}  // namespace spg
