// Gradients of a loss L with dL/dC = G on C's stored entries, with respect to
// the stored values of A and B (sparsity patterns fixed). Both are sampled
// sparse products over the same product space as the forward pass:
//   dB(k,j) = sum over stored A(i,k), in A's storage order, of A(i,k) G(i,j)
//   dA(i,k) = sum over stored B(k,j), j ascending,          of G(i,j) B(k,j)
// One thread owns one output entry and adds its terms sequentially in the
// stated order (no fused multiply-add), so the result is reproducible and
// matches a plain sequential loop bit for bit.
//
// Every term is one product of the forward pass: stored B entry t of column j
// times the u-th entry of A's column bri[t]. A view built once per plan
// records that product's rank among the entries of C's column j (dst, by a
// binary search of C's sorted rows), so G(i,j) sits at ccp[j] + rank; it also
// holds, per stored B entry, its first product (pofs) and its column's first C
// entry (cb); per stored A entry, its column and offset in it; and a row view
// of B (entries of each row by ascending column) with the same two values per
// entry, so the dA loop reads them without an indirection.
#include "devutil.h"

namespace spg {

// largest j in [0, n) with cp[j] <= t (columns may be empty)
__device__ __forceinline__ int column_of(const int32_t *cp, int n, int t) {
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (cp[mid] <= t) lo = mid;
        else hi = mid;
    }
    return lo;
}

constexpr int kBwUnroll = 4;  // terms whose loads are issued together

template <typename V>
__device__ __forceinline__ V g_at(const V *__restrict__ gv, long long nnzc, int cb, uint32_t d,
                                  int &bad) {
    const long long gp = (long long)cb + (long long)(d & ~kDstLater);
    if (gp >= nnzc) { bad = 1; return V(0); }
    return gv[gp];
}

template <typename V>
__device__ __forceinline__ void grad_b(const BwView &w, int t, const V *__restrict__ av,
                                       const V *__restrict__ gv, V *__restrict__ db, int *err) {
    const int2 e = w.E[t];  // A column start and length of the entry's row of B
    const long long base = w.pofs[t];
    const int cb = w.cb[t];
    const V *__restrict__ ap = av + e.x;
    const uint32_t *__restrict__ dp = w.dst + base;
    V acc = V(0);
    int bad = 0, u = 0;
    for (; u + kBwUnroll <= e.y; u += kBwUnroll) {
        V a[kBwUnroll], g[kBwUnroll];
        uint32_t d[kBwUnroll];
#pragma unroll
        for (int v = 0; v < kBwUnroll; ++v) {
            a[v] = ap[u + v];
            d[v] = dp[u + v];
        }
#pragma unroll
        for (int v = 0; v < kBwUnroll; ++v) g[v] = g_at(gv, w.nnzc, cb, d[v], bad);
#pragma unroll
        for (int v = 0; v < kBwUnroll; ++v) acc = acc + a[v] * g[v];
    }
    for (; u < e.y; ++u) acc = acc + ap[u] * g_at(gv, w.nnzc, cb, dp[u], bad);
    db[t] = acc;
    if (bad) atomicOr(err, ERR_CSC);
}

template <typename V>
__device__ __forceinline__ void grad_a(const BwView &w, int q, const V *__restrict__ bv,
                                       const V *__restrict__ gv, V *__restrict__ da, int *err) {
    const int2 ku = w.aview[q];  // column of A (= row of B) and offset in that column
    const int r0 = w.rowptr[ku.x], r1 = w.rowptr[ku.x + 1];
    V acc = V(0);
    int bad = 0, r = r0;
    for (; r + kBwUnroll <= r1; r += kBwUnroll) {
        int2 tc[kBwUnroll];
        long long pf[kBwUnroll];
#pragma unroll
        for (int v = 0; v < kBwUnroll; ++v) {
            tc[v] = w.rv[r + v];
            pf[v] = w.rvp[r + v];
        }
        uint32_t d[kBwUnroll];
        V b[kBwUnroll], g[kBwUnroll];
#pragma unroll
        for (int v = 0; v < kBwUnroll; ++v) {
            d[v] = w.dst[pf[v] + ku.y];
            b[v] = bv[tc[v].x];
        }
#pragma unroll
        for (int v = 0; v < kBwUnroll; ++v) g[v] = g_at(gv, w.nnzc, tc[v].y, d[v], bad);
#pragma unroll
        for (int v = 0; v < kBwUnroll; ++v) acc = acc + g[v] * b[v];
    }
    for (; r < r1; ++r) {
        const int2 tc = w.rv[r];
        const uint32_t d = w.dst[w.rvp[r] + ku.y];
        acc = acc + g_at(gv, w.nnzc, tc.y, d, bad) * bv[tc.x];
    }
    da[q] = acc;
    if (bad) atomicOr(err, ERR_CSC);
}

// Both gradients in one launch: workgroups [0, nbw) take dB (one thread per
// stored B entry), the rest dA (one thread per stored A entry).
template <typename V>
__global__ __launch_bounds__(kBlock) void k_grad(BwView w, int nnza, int nnzb, int nbw,
                                                 const V *__restrict__ av,
                                                 const V *__restrict__ bv,
                                                 const V *__restrict__ gv, V *__restrict__ da,
                                                 V *__restrict__ db, int *err) {
    if ((int)blockIdx.x < nbw) {
        const int t = blockIdx.x * kBlock + threadIdx.x;
        if (t < nnzb) grad_b<V>(w, t, av, gv, db, err);
    } else {
        const int q = (blockIdx.x - nbw) * kBlock + threadIdx.x;
        if (q < nnza) grad_a<V>(w, q, bv, gv, da, err);
    }
}

// ---------------------------------------------------------------- view construction
// per stored B entry: its column, its column's first C entry, the length of
// the A column it selects, and the count of its row
__global__ __launch_bounds__(kBlock) void k_bv_bent(Prob p, const int2 *__restrict__ E,
                                                    int32_t *bcol, int32_t *cb, int32_t *len,
                                                    int32_t *cnt) {
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= p.nnzb) return;
    const int j = column_of(p.bcp, p.n, t);
    bcol[t] = j;
    cb[t] = p.ccp[j];
    len[t] = E[t].y;
    atomicAdd(&cnt[p.bri[t]], 1);
}

// per stored A entry: its column and its offset in the column
__global__ __launch_bounds__(kBlock) void k_bv_aent(Prob p, int2 *aview) {
    const int q = blockIdx.x * kBlock + threadIdx.x;
    if (q >= p.nnza) return;
    const int k = column_of(p.acp, p.k, q);
    aview[q] = make_int2(k, q - p.acp[k]);
}

__global__ __launch_bounds__(kBlock) void k_bv_fill(Prob p, const int32_t *rowptr,
                                                    const int32_t *bcol, int32_t *fill,
                                                    int32_t *colj, int32_t *pos) {
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= p.nnzb) return;
    const int k = p.bri[t];
    const int slot = rowptr[k] + atomicAdd(&fill[k], 1);
    colj[slot] = bcol[t];
    pos[slot] = t;
}

// each row's entries by ascending column (Shell sort with Ciura's gaps)
__global__ __launch_bounds__(kBlock) void k_bv_sort(int nrows, const int32_t *rowptr,
                                                    int32_t *colj, int32_t *pos) {
    const int k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= nrows) return;
    const int b = rowptr[k], e = rowptr[k + 1], len = e - b;
    const int gaps[8] = {701, 301, 132, 57, 23, 10, 4, 1};
    for (int gi = 0; gi < 8; ++gi) {
        const int gap = gaps[gi];
        if (gap >= len) continue;
        for (int u = b + gap; u < e; ++u) {
            const int cj = colj[u], cp = pos[u];
            int v = u;
            while (v - gap >= b && colj[v - gap] > cj) {
                colj[v] = colj[v - gap];
                pos[v] = pos[v - gap];
                v -= gap;
            }
            colj[v] = cj;
            pos[v] = cp;
        }
    }
}

// the row view's per-entry values: (B entry, C column start) and first product
__global__ __launch_bounds__(kBlock) void k_bv_pack(int nnzb, const int32_t *pos,
                                                    const int32_t *cb, const long long *pofs,
                                                    int2 *rv, long long *rvp) {
    const int r = blockIdx.x * kBlock + threadIdx.x;
    if (r >= nnzb) return;
    const int t = pos[r];
    rv[r] = make_int2(t, cb[t]);
    rvp[r] = pofs[t];
}

// rank of every product's row inside its C column (C's rows are ascending:
// a binary search), thread per stored B entry walking its A column
__global__ __launch_bounds__(kBlock) void k_bv_dst(Prob p, const int2 *__restrict__ E,
                                                   const long long *__restrict__ pofs,
                                                   const int32_t *__restrict__ bcol,
                                                   const int32_t *__restrict__ cri,
                                                   uint32_t *__restrict__ dst, int *err) {
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= p.nnzb) return;
    const int j = bcol[t];
    const int c0 = p.ccp[j], c1 = p.ccp[j + 1];
    const int2 e = E[t];
    const long long base = pofs[t];
    int bad = 0;
    for (int u = 0; u < e.y; ++u) {
        const int row = p.ari[e.x + u];
        int lo = c0, hi = c1;  // first position whose row is not below `row`
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (cri[mid] < row) lo = mid + 1;
            else hi = mid;
        }
        if (lo >= c1 || cri[lo] != row) {  // C does not hold the product's row
            bad = 1;
            dst[base + u] = 0;
        } else {
            dst[base + u] = (uint32_t)(lo - c0);
        }
    }
    if (bad) atomicOr(err, ERR_CSC);
}

hipError_t launch_bw_dst(const Prob &p, const int2 *E, const long long *pofs, const int32_t *bcol,
                         const int32_t *cri, uint32_t *dst, int *err, hipStream_t s) {
    if (p.nnzb <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_bv_dst, dim3(ceil_div(p.nnzb, kBlock)), dim3(kBlock), 0, s, p, E, pofs,
                       bcol, cri, dst, err);
    return hipGetLastError();
}

// ---------------------------------------------------------------- launchers
hipError_t launch_bw_view(const Prob &p, const int2 *E, const BwBuild &b, BwView &w,
                          hipStream_t s) {
    const int nrows = p.k;  // rows of B
    hipError_t e = hipMemsetAsync(b.rowptr, 0, sizeof(int32_t) * (size_t)(nrows + 1), s);
    if (e != hipSuccess) return e;
    e = hipMemsetAsync(b.fill, 0, sizeof(int32_t) * (size_t)(nrows > 0 ? nrows : 1), s);
    if (e != hipSuccess) return e;
    const int gb = ceil_div(p.nnzb, kBlock);
    if (gb > 0)
        hipLaunchKernelGGL(k_bv_bent, dim3(gb), dim3(kBlock), 0, s, p, E, b.bcol, b.cb, b.len,
                           b.rowptr);
    if (p.nnza > 0)
        hipLaunchKernelGGL(k_bv_aent, dim3(ceil_div(p.nnza, kBlock)), dim3(kBlock), 0, s, p,
                           b.aview);
    e = launch_scan_i32(b.rowptr, nrows + 1, b.scratch, b.nscratch, b.rowptr, s);
    if (e != hipSuccess) return e;
    e = launch_scan_i64(b.len, p.nnzb, b.scratch2, b.nscratch2, b.pofs, s);
    if (e != hipSuccess) return e;
    if (gb > 0)
        hipLaunchKernelGGL(k_bv_fill, dim3(gb), dim3(kBlock), 0, s, p, (const int32_t *)b.rowptr,
                           (const int32_t *)b.bcol, b.fill, b.colj, b.pos);
    if (nrows > 0)
        hipLaunchKernelGGL(k_bv_sort, dim3(ceil_div(nrows, kBlock)), dim3(kBlock), 0, s, nrows,
                           (const int32_t *)b.rowptr, b.colj, b.pos);
    if (gb > 0)
        hipLaunchKernelGGL(k_bv_pack, dim3(gb), dim3(kBlock), 0, s, p.nnzb,
                           (const int32_t *)b.pos, (const int32_t *)b.cb,
                           (const long long *)b.pofs, b.rv, b.rvp);
    w.E = E;
    w.dst = b.dst;
    w.pofs = b.pofs;
    w.cb = b.cb;
    w.aview = b.aview;
    w.rowptr = b.rowptr;
    w.rv = b.rv;
    w.rvp = b.rvp;
    return hipGetLastError();
}

hipError_t launch_backward(const Prob &p, const BwView &w, bool f64, const void *av,
                           const void *bv, const void *gv, void *da, void *db, int *err,
                           hipStream_t s) {
    const int nbw = (db && p.nnzb > 0) ? ceil_div(p.nnzb, kBlock) : 0;
    const int naw = (da && p.nnza > 0) ? ceil_div(p.nnza, kBlock) : 0;
    if (nbw + naw == 0) return hipSuccess;
    if (f64)
        hipLaunchKernelGGL(k_grad<double>, dim3(nbw + naw), dim3(kBlock), 0, s, w, p.nnza, p.nnzb,
                           nbw, (const double *)av, (const double *)bv, (const double *)gv,
                           (double *)da, (double *)db, err);
    else
        hipLaunchKernelGGL(k_grad<float>, dim3(nbw + naw), dim3(kBlock), 0, s, w, p.nnza, p.nnzb,
                           nbw, (const float *)av, (const float *)bv, (const float *)gv,
                           (float *)da, (float *)db, err);
    return hipGetLastError();
}

}  // namespace spg
