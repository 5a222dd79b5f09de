// Product expansion, tiles, window offsets, and the numeric phase.
//
// Product-balanced tiles: tile t holds the columns whose first product lies in
// [t * kProdTile, (t + 1) * kProdTile) of the product space, so every tile has
// about kProdTile products (plus the tail of its last column).
//
// Expansion: one workgroup per tile walks the tile's stored B entries in
// storage order (they are contiguous) and writes the row of every product --
// the rows of the A column each entry selects, in storage order -- to the
// product space. This is the only pass that expands the products of
// Gustavson's column method (Section 2.1) from the inputs' index arrays; the
// symbolic accumulators stream these rows.
//
// Numeric: the symbolic phase left, per product, a destination (the rank of
// its output row, or for a product that is not the first of its output entry
// a place in the list of such "later" products with its occurrence index k),
// and, for columns of at most kSortMax products without row windows, the
// output order (the first product and the row of every output entry). One
// workgroup per tile forms the products A(i,k) * B(k,j) of its columns of at
// most kOrderMax products from coalesced reads of the selected A columns into
// LDS, then writes their output entries in order as 0 + first product. Larger
// or windowed columns are done by one workgroup per column through the
// destinations. Later products are staged; layer
// kernels add those of occurrence index 1, 2, ... in that order, so every
// output entry is summed in Algorithm 1's order and rounding, bit for bit.
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

__global__ __launch_bounds__(kBlock) void k_expand(KArgs a) {
    constexpr int PER = 4;
    __shared__ ExpSmem S;
    if (a.hdr->err) return;
    const int tid = threadIdx.x;
    const int g0 = a.tilestart[blockIdx.x], g1 = a.tilestart[blockIdx.x + 1];
    int *__restrict__ prow = a.prow;
    int bad = 0;
    for_each_segment(a, g0, g1, [&](int, const Prob &d, int j0, int j1) {
        long long base = a.colprod[d.col0 + j0];
        const int pb = d.bcp[j0], pe = d.bcp[j1];  // checked by the classification
        const int2 *__restrict__ Ep = a.E + d.ebase;
        const int *__restrict__ ari = d.ari;
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
    });
    if (bad) atomicOr(&a.hdr->err, ERR_CSC);
}

hipError_t launch_expand(const KArgs &a, hipStream_t s) {
    if (a.nptiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_expand, dim3(a.nptiles), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------- numeric, tiles
constexpr int kColWin = 256;                   // columns per window of a tile
constexpr int kStage = kProdTile + kOrderMax;  // staged products of a tile

// the tiles write a column in output order when it has at most kOrderMax
// products and no row windows (its output order is then recorded)
__device__ __forceinline__ bool has_order(int op, int binw) {
    return op <= kOrderMax && (binw >> 8) <= 1;
}

template <typename V>
struct NumSmem {
    V val[kStage];           // products of the tile's ordered columns (by product offset)
    int s_acp[kBlock];       // A column start of each stored B entry of the B window
    int s_eoff[kBlock];      // first product of each stored B entry of the B window
    int s_col[kBlock];       // window column of each stored B entry of the B window
    V s_bv[kBlock];          // B value of each stored B entry of the B window
    int s_bcp[kColWin + 1];  // B column pointers of the column window
    int s_c0[kColWin + 1];   // C column pointers of the column window
    int s_pb[kColWin + 1];   // first product of each column, relative to the tile
    int s_ok[kColWin];       // column written in output order
    int scan_tmp[kBlock / 64 + 1];
};

template <typename V>
__global__ __launch_bounds__(kBlock) void k_numeric(KArgs a) {
    constexpr int PER = 4;   // products per thread per chunk
    constexpr int OPER = 8;  // output entries per thread per chunk
    __shared__ NumSmem<V> S;
    if (a.hdr->err) return;
    const int tid = threadIdx.x;
    const int g0 = a.tilestart[blockIdx.x], g1 = a.tilestart[blockIdx.x + 1];
    if (g0 >= g1) return;
    const long long tbase = a.colprod[g0];
    V *__restrict__ lv = (V *)a.lv;
    int bad = 0;
    for_each_segment(a, g0, g1, [&](int pid, const Prob &d, int js, int je) {
        const int2 *__restrict__ Ep = a.E + d.ebase;
        const V *__restrict__ av = (const V *)d.av;
        const V *__restrict__ bv = (const V *)d.bv;
        int *__restrict__ cri = d.cri;
        V *__restrict__ cv = (V *)d.cv;
        for (int jw = js; jw < je; jw += kColWin) {
            const int nc = min(kColWin, je - jw);
            const int gw = d.col0 + jw;
            for (int c = tid; c <= nc; c += kBlock) {
                S.s_bcp[c] = d.bcp[jw + c];
                S.s_c0[c] = d.ccp[jw + c];
                const long long pc = c < nc ? a.colprod[gw + c]
                                            : a.colprod[gw + nc - 1] + a.op[gw + nc - 1];
                S.s_pb[c] = (int)(pc - tbase);
                if (c < nc) S.s_ok[c] = has_order(a.op[gw + c], a.binw[gw + c]);
            }
            __syncthreads();
            // ---- products of the window's ordered columns into LDS; later
            // products staged for the layer kernels. The next B window's
            // loads are issued before the current one is processed.
            long long base = tbase + S.s_pb[0];
            const int pb = S.s_bcp[0], pe = S.s_bcp[nc];
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
                int z = 0, acp = 0, col = 0;
                V b = V(0);
                if (t < pe) {
                    col = last_le(S.s_bcp, nc + 1, t);
                    z = ez.y;
                    if (S.s_ok[col]) {
                        acp = ez.x;
                        b = b0;
                    }
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
                    V v[PER];
                    uint32_t dc[PER];
                    int c[PER];
#pragma unroll
                    for (int u = 0; u < PER; ++u) {
                        const int e = e0 + u * kBlock + tid;
                        c[u] = -1;
                        if (e < Ew) {
                            const int tt = last_le(S.s_eoff, nbw, e);
                            if (S.s_ok[S.s_col[tt]]) {
                                c[u] = S.s_col[tt];
                                const int q = S.s_acp[tt] + e - S.s_eoff[tt];
                                v[u] = av[q] * S.s_bv[tt];
                                dc[u] = a.dst[base + e];
                            }
                        }
                    }
#pragma unroll
                    for (int u = 0; u < PER; ++u) {
                        if (c[u] < 0) continue;
                        const long long eg = base + e0 + u * kBlock + tid;
                        S.val[eg - tbase] = v[u];
                        if (dc[u] & kDstLater) {
                            const int li = (int)(dc[u] & ~kDstLater);
                            if (li >= a.later_cap) { bad = 1; continue; }
                            const int o = a.lr[li];
                            if (o < 0 || o >= S.s_c0[c[u] + 1] - S.s_c0[c[u]]) { bad = 1; continue; }
                            a.lo[li] = S.s_c0[c[u]] + o;
                            a.lpid[li] = pid;
                            lv[li] = v[u];
                        }
                    }
                }
                base += Ew;
                __syncthreads();
            }
            // ---- output entries of the window's ordered columns, in order
            const int o0 = S.s_c0[0], o1 = S.s_c0[nc];
            for (int oc = o0; oc < o1; oc += OPER * kBlock) {
                int c[OPER], e[OPER], row[OPER];
#pragma unroll
                for (int u = 0; u < OPER; ++u) {
                    const int o = oc + u * kBlock + tid;
                    c[u] = -1;
                    if (o < o1) {
                        const int cc = last_le(S.s_c0, nc + 1, o);
                        if (S.s_ok[cc]) {
                            c[u] = cc;
                            const long long po = tbase + S.s_pb[cc] + (o - S.s_c0[cc]);
                            e[u] = a.perm[po];
                            row[u] = a.crow[po];
                        }
                    }
                }
#pragma unroll
                for (int u = 0; u < OPER; ++u) {
                    if (c[u] < 0) continue;
                    if (e[u] < 0 || e[u] >= S.s_pb[c[u] + 1] - S.s_pb[c[u]]) {
                        bad = 1;
                        continue;
                    }
                    const int o = oc + u * kBlock + tid;
                    cri[o] = row[u];
                    cv[o] = V(0) + S.val[S.s_pb[c[u]] + e[u]];
                }
            }
            __syncthreads();
        }
    });
    if (bad) atomicOr(&a.hdr->err, ERR_GROUP);
}

// ---------------------------------------------------------------- numeric, other columns
template <typename V>
struct BigSmem {
    int s_acp[kBlock];
    int s_eoff[kBlock];
    V s_bv[kBlock];
    int scan_tmp[kBlock / 64 + 1];
};

template <typename V>
__global__ __launch_bounds__(kBlock) void k_numeric_big(KArgs a, int first, int n) {
    constexpr int PER = 4;
    __shared__ BigSmem<V> S;
    if (a.hdr->err) return;
    const int tid = threadIdx.x;
    V *__restrict__ lv = (V *)a.lv;
    for (int li0 = blockIdx.x; li0 < n; li0 += gridDim.x) {
        const int4 ent = a.binlist[first + li0];
        const int g = ent.x, bs = ent.y, be = ent.y + ent.z;
        const int bwin = a.binw[g];
        if (has_order(a.op[g], bwin)) continue;  // done by the tiles
        const int pid = find_prob(a, g);
        const Prob d = get_prob(a, pid);
        const int j = g - d.col0;
        const int W = max(bwin >> 8, 1);
        const int it0 = W > 1 ? a.colitem[g] : 0;
        long long base = a.colprod[g];
        const int c0 = d.ccp[j], clen = d.ccp[j + 1] - c0;
        const int2 *__restrict__ Ep = a.E + d.ebase;
        const V *__restrict__ av = (const V *)d.av;
        const V *__restrict__ bv = (const V *)d.bv;
        int *__restrict__ cri = d.cri + c0;
        V *__restrict__ cv = (V *)d.cv + c0;
        int bad = 0;
        for (int bw = bs; bw < be; bw += kBlock) {
            const int t = bw + tid;
            int z = 0, acp = 0;
            V b = V(0);
            if (t < be) {
                const int2 ez = Ep[t];
                acp = ez.x;
                z = ez.y;
                b = bv[t];
            }
            int Ew;
            const int ex = block_excl_scan(z, S.scan_tmp, Ew);
            S.s_acp[tid] = acp;
            S.s_eoff[tid] = ex;
            S.s_bv[tid] = b;
            __syncthreads();
            const int nbw = min(kBlock, be - bw);
            for (int e0 = 0; e0 < Ew; e0 += PER * kBlock) {
                int row[PER];
                V v[PER];
                uint32_t dc[PER];
#pragma unroll
                for (int u = 0; u < PER; ++u) {
                    const int e = e0 + u * kBlock + tid;
                    row[u] = -1;
                    if (e < Ew) {
                        const int tt = last_le(S.s_eoff, nbw, e);
                        const int q = S.s_acp[tt] + e - S.s_eoff[tt];
                        row[u] = a.prow[base + e];
                        v[u] = av[q] * S.s_bv[tt];
                        dc[u] = a.dst[base + e];
                    }
                }
#pragma unroll
                for (int u = 0; u < PER; ++u) {
                    if (row[u] < 0) continue;
                    const bool later = (dc[u] & kDstLater) != 0;
                    const int li = (int)(dc[u] & ~kDstLater);
                    if (later && li >= a.later_cap) { bad = 1; continue; }
                    int o = later ? a.lr[li] : li;
                    if (W > 1) o += a.itemoff[it0 + window_of(row[u], W, d.m)];
                    if (o < 0 || o >= clen) { bad = 1; continue; }
                    if (!later) {
                        cri[o] = row[u];
                        cv[o] = V(0) + v[u];
                    } else {
                        a.lo[li] = c0 + o;
                        a.lpid[li] = pid;
                        lv[li] = v[u];
                    }
                }
            }
            base += Ew;
            __syncthreads();
        }
        if (bad) atomicOr(&a.hdr->err, ERR_GROUP);
    }
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
    if (a.nptiles <= 0) return hipSuccess;
    if (f64) hipLaunchKernelGGL((k_numeric<double>), dim3(a.nptiles), dim3(kBlock), 0, s, a);
    else hipLaunchKernelGGL((k_numeric<float>), dim3(a.nptiles), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_numeric_big(const KArgs &a, bool f64, int first, int nbig, hipStream_t s) {
    if (nbig <= 0) return hipSuccess;
    if (f64)
        hipLaunchKernelGGL((k_numeric_big<double>), dim3(nbig), dim3(kBlock), 0, s, a, first, nbig);
    else
        hipLaunchKernelGGL((k_numeric_big<float>), dim3(nbig), dim3(kBlock), 0, s, a, first, nbig);
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
