// Product expansion, window offsets, and the numeric phase.
//
// Expansion: one workgroup per tile of columns walks the tile's stored B
// entries in storage order (they are contiguous), and writes the row of
// every product -- the rows of the A column each entry selects, in storage
// order -- to the product space. This is the only pass that expands the
// products of Gustavson's column method (Section 2.1) from the inputs'
// index arrays; the symbolic accumulators stream these rows.
//
// Numeric: the symbolic phase left a destination per product: the rank of its
// output row inside its column (or row window), or, for a product that is not
// the first of its output entry, its place in a list of such "later"
// products together with its occurrence index k. The numeric phase walks the
// tiles the same way, forms every product A(i,k) * B(k,j) from coalesced
// reads of the selected A columns, writes every first product as 0 + product
// to its output position, and stages the later ones. Layer kernels then add
// the staged products of occurrence index 1, 2, ... in that order, so every
// output entry is summed in Algorithm 1's order and rounding, bit for bit.
#include "devutil.h"

namespace spg {

__device__ __forceinline__ void tile_of(const KArgs &a, int &pid, int &j0, int &j1) {
    if (a.nprob == 1) {
        pid = 0;
        j0 = blockIdx.x * kTile;
        j1 = min(a.single.n, j0 + kTile);
    } else {
        const int4 tl = a.tiles[blockIdx.x];
        pid = tl.x;
        j0 = tl.y;
        j1 = tl.z;
    }
}

// ---------------------------------------------------------------- expansion
struct ExpSmem {
    int s_acp[kBlock];   // A column start of each stored B entry of the B window
    int s_eoff[kBlock];  // first product of each stored B entry of the B window
    int scan_tmp[kBlock / 64 + 1];
};

__global__ __launch_bounds__(kBlock) void k_expand(KArgs a) {
    constexpr int PER = 4;
    __shared__ ExpSmem S;
    if (a.hdr->err) return;
    int pid, j0, j1;
    tile_of(a, pid, j0, j1);
    const Prob d = get_prob(a, pid);
    const int tid = threadIdx.x;
    long long base = a.colprod[d.col0 + j0];
    const int pb = d.bcp[j0], pe = d.bcp[j1];  // checked by the classification
    const int2 *__restrict__ Ep = a.E + d.ebase;
    const int *__restrict__ ari = d.ari;
    int *__restrict__ prow = a.prow;
    int bad = 0;
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
                    bad = 1;
                    row = 0;
                }
                prow[base + e] = row;
            }
        }
        base += Ew;
        __syncthreads();
    }
    if (bad) atomicOr(&a.hdr->err, ERR_CSC);
}

hipError_t launch_expand(const KArgs &a, hipStream_t s) {
    if (a.ntiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_expand, dim3(a.ntiles), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------- window offsets
// one thread per hash column: exclusive prefix of its windows' distinct rows
__global__ __launch_bounds__(kBlock) void k_item_offsets(KArgs a, int first, int n) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int g = a.binlist[first + i].x;
    const int W = a.binw[g] >> 8;
    const int it0 = a.colitem[g];
    int run = 0;
    for (int w = 0; w < W; ++w) {
        const int c = a.itemcnt[it0 + w];
        a.itemoff[it0 + w] = run;
        run += c;
    }
}

hipError_t launch_item_offsets(const KArgs &a, int first, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_item_offsets, dim3(ceil_div(n, kBlock)), dim3(kBlock), 0, s, a, first, n);
    return hipGetLastError();
}

// ---------------------------------------------------------------- numeric
template <typename V>
struct NumSmem {
    int s_acp[kBlock];       // A column start of each stored B entry of the B window
    int s_eoff[kBlock];      // first product of each stored B entry of the B window
    int s_col[kBlock];       // tile column of each stored B entry of the B window
    V s_bv[kBlock];          // B value of each stored B entry of the B window
    int s_bcp[kTile + 1];    // B column pointers of the tile
    int s_c0[kTile + 1];     // C column pointers of the tile
    int s_w[kTile];          // row windows of each tile column (0 or 1: whole column)
    int s_it0[kTile];        // first work item of each windowed tile column
    int scan_tmp[kBlock / 64 + 1];
};

template <typename V>
__global__ __launch_bounds__(kBlock) void k_numeric(KArgs a) {
    constexpr int PER = 2;
    __shared__ NumSmem<V> S;
    if (a.hdr->err) return;
    int pid, j0, j1;
    tile_of(a, pid, j0, j1);
    const Prob d = get_prob(a, pid);
    const int tid = threadIdx.x;
    const int nt = j1 - j0;
    const int g0 = d.col0 + j0;
    for (int c = tid; c <= nt; c += kBlock) {
        S.s_bcp[c] = d.bcp[j0 + c];
        S.s_c0[c] = d.ccp[j0 + c];
    }
    for (int c = tid; c < nt; c += kBlock) {
        const int W = a.binw[g0 + c] >> 8;
        S.s_w[c] = W;
        S.s_it0[c] = W > 1 ? a.colitem[g0 + c] : 0;
    }
    __syncthreads();
    long long base = a.colprod[g0];
    const int pb = S.s_bcp[0], pe = S.s_bcp[nt];
    const int2 *__restrict__ Ep = a.E + d.ebase;
    const int *__restrict__ ari = d.ari;
    const V *__restrict__ av = (const V *)d.av;
    const V *__restrict__ bv = (const V *)d.bv;
    int *__restrict__ cri = d.cri;
    V *__restrict__ cv = (V *)d.cv;
    V *__restrict__ lv = (V *)a.lv;
    int bad = 0;
    for (int bw = pb; bw < pe; bw += kBlock) {
        const int t = bw + tid;
        int z = 0, acp = 0, col = 0;
        V b = V(0);
        if (t < pe) {
            const int2 ez = Ep[t];
            acp = ez.x;
            z = ez.y;
            b = bv[t];
            col = last_le(S.s_bcp, nt + 1, t);
        }
        int Ew;
        const int ex = block_excl_scan(z, S.scan_tmp, Ew);
        S.s_acp[tid] = acp;
        S.s_eoff[tid] = ex;
        S.s_col[tid] = col;
        S.s_bv[tid] = b;
        __syncthreads();
        const int nbw = min(kBlock, pe - bw);
        for (int e0 = 0; e0 < Ew; e0 += PER * kBlock) {
            int row[PER], tt[PER];
            V val[PER];
            uint32_t dc[PER];
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                const int e = e0 + u * kBlock + tid;
                row[u] = -1;
                if (e < Ew) {
                    tt[u] = last_le(S.s_eoff, nbw, e);
                    const int q = S.s_acp[tt[u]] + e - S.s_eoff[tt[u]];
                    row[u] = ari[q];
                    val[u] = av[q] * S.s_bv[tt[u]];
                    dc[u] = a.dst[base + e];
                }
            }
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                if (row[u] < 0) continue;
                const int c = S.s_col[tt[u]];
                const int c0 = S.s_c0[c], clen = S.s_c0[c + 1] - c0;
                const bool later = (dc[u] & kDstLater) != 0;
                const int li = (int)(dc[u] & ~kDstLater);
                if (later && li >= a.later_cap) {  // destinations do not match the plan
                    bad = 1;
                    continue;
                }
                int o = later ? a.lr[li] : li;
                const int W = S.s_w[c];
                if (W > 1) o += a.itemoff[S.s_it0[c] + window_of(row[u], W, d.m)];
                if (o < 0 || o >= clen || row[u] >= d.m) {
                    bad = 1;
                    continue;
                }
                if (!later) {
                    cri[c0 + o] = row[u];
                    cv[c0 + o] = V(0) + val[u];
                } else {
                    a.lo[li] = c0 + o;
                    a.lpid[li] = pid;
                    lv[li] = val[u];
                }
            }
        }
        base += Ew;
        __syncthreads();
    }
    if (bad) atomicOr(&a.hdr->err, ERR_GROUP);
}

// later products of occurrence index k, added to their (already written)
// output entries; every entry has at most one product of each index
template <typename V>
__global__ __launch_bounds__(kBlock) void k_layer(KArgs a, int k, long long n) {
    const V *__restrict__ lv = (const V *)a.lv;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n;
         i += (long long)gridDim.x * kBlock) {
        if (a.lk[i] != k) continue;
        const Prob d = get_prob(a, a.lpid[i]);
        V *cv = (V *)d.cv;
        const int o = a.lo[i];
        cv[o] = cv[o] + lv[i];
    }
}

hipError_t launch_numeric(const KArgs &a, bool f64, hipStream_t s) {
    if (a.ntiles <= 0) return hipSuccess;
    if (f64) hipLaunchKernelGGL((k_numeric<double>), dim3(a.ntiles), dim3(kBlock), 0, s, a);
    else hipLaunchKernelGGL((k_numeric<float>), dim3(a.ntiles), dim3(kBlock), 0, s, a);
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
