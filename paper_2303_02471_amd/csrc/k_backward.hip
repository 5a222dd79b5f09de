// Gradients of a loss L with dL/dC = G on C's stored entries, with respect to
// the stored values of A and B (sparsity patterns fixed). Both are sampled
// sparse products over the same product space as the forward pass:
//   dB(k,j) = sum over stored A(i,k), in A's storage order, of A(i,k) G(i,j)
//   dA(i,k) = sum over stored B(k,j), j ascending,          of G(i,j) B(k,j)
// One thread owns one output entry and adds its terms sequentially in the
// stated order (no fused multiply-add), so the result is reproducible and
// matches a plain sequential loop bit for bit. G(i,j) is found by binary
// search of row i in the ascending rows of C's column j. dA walks B by rows
// through a row view of B's pattern (built once per plan).
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

// position of row i in cri[c0, c1) (ascending), or -1
__device__ __forceinline__ int find_row(const int32_t *cri, int c0, int c1, int i) {
    int lo = c0, hi = c1;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (cri[mid] < i) lo = mid + 1;
        else hi = mid;
    }
    return (lo < c1 && cri[lo] == i) ? lo : -1;
}

template <typename V>
__global__ __launch_bounds__(kBlock) void k_grad_b(Prob p, const V *__restrict__ av,
                                                   const int32_t *__restrict__ cri,
                                                   const V *__restrict__ gv, V *__restrict__ db,
                                                   int *err) {
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= p.nnzb) return;
    const int j = column_of(p.bcp, p.n, t);
    const int k = p.bri[t];
    const int c0 = p.ccp[j], c1 = p.ccp[j + 1];
    V acc = V(0);
    for (int q = p.acp[k]; q < p.acp[k + 1]; ++q) {
        const int at = find_row(cri, c0, c1, p.ari[q]);
        if (at < 0) { atomicOr(err, ERR_CSC); break; }
        acc = acc + av[q] * gv[at];
    }
    db[t] = acc;
}

template <typename V>
__global__ __launch_bounds__(kBlock) void k_grad_a(Prob p, const V *__restrict__ bv,
                                                   const int32_t *__restrict__ cri,
                                                   const V *__restrict__ gv, V *__restrict__ da,
                                                   const int32_t *__restrict__ rowptr,
                                                   const int32_t *__restrict__ colj,
                                                   const int32_t *__restrict__ pos, int *err) {
    const int q = blockIdx.x * kBlock + threadIdx.x;
    if (q >= p.nnza) return;
    const int k = column_of(p.acp, p.k, q);
    const int i = p.ari[q];
    V acc = V(0);
    for (int r = rowptr[k]; r < rowptr[k + 1]; ++r) {
        const int j = colj[r];
        const int at = find_row(cri, p.ccp[j], p.ccp[j + 1], i);
        if (at < 0) { atomicOr(err, ERR_CSC); break; }
        acc = acc + gv[at] * bv[pos[r]];
    }
    da[q] = acc;
}

// ---------------------------------------------------------------- row view of B
__global__ __launch_bounds__(kBlock) void k_bt_count(Prob p, int32_t *cnt) {
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t < p.nnzb) atomicAdd(&cnt[p.bri[t]], 1);
}

__global__ __launch_bounds__(kBlock) void k_bt_fill(Prob p, const int32_t *rowptr, int32_t *fill,
                                                    int32_t *colj, int32_t *pos) {
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= p.nnzb) return;
    const int j = column_of(p.bcp, p.n, t);
    const int k = p.bri[t];
    const int slot = rowptr[k] + atomicAdd(&fill[k], 1);
    colj[slot] = j;
    pos[slot] = t;
}

// each row's entries by ascending column (Shell sort with Ciura's gaps)
__global__ __launch_bounds__(kBlock) void k_bt_sort(int nrows, const int32_t *rowptr,
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

// ---------------------------------------------------------------- launchers
hipError_t launch_btranspose(const Prob &p, int32_t *rowptr, int32_t *fill, int32_t *colj,
                             int32_t *pos, long long *scratch, int nscratch, hipStream_t s) {
    const int nrows = p.k;  // rows of B
    hipError_t e = hipMemsetAsync(rowptr, 0, sizeof(int32_t) * (size_t)(nrows + 1), s);
    if (e != hipSuccess) return e;
    e = hipMemsetAsync(fill, 0, sizeof(int32_t) * (size_t)(nrows > 0 ? nrows : 1), s);
    if (e != hipSuccess) return e;
    const int gb = ceil_div(p.nnzb, kBlock);
    if (gb > 0) hipLaunchKernelGGL(k_bt_count, dim3(gb), dim3(kBlock), 0, s, p, rowptr);
    e = launch_scan_i32(rowptr, nrows + 1, scratch, nscratch, rowptr, s);
    if (e != hipSuccess) return e;
    if (gb > 0) hipLaunchKernelGGL(k_bt_fill, dim3(gb), dim3(kBlock), 0, s, p,
                                   (const int32_t *)rowptr, fill, colj, pos);
    if (nrows > 0)
        hipLaunchKernelGGL(k_bt_sort, dim3(ceil_div(nrows, kBlock)), dim3(kBlock), 0, s, nrows,
                           (const int32_t *)rowptr, colj, pos);
    return hipGetLastError();
}

hipError_t launch_backward(const Prob &p, bool f64, const void *av, const void *bv,
                           const int32_t *cri, const void *gv, void *da, void *db,
                           const int32_t *rowptr, const int32_t *colj, const int32_t *pos,
                           int *err, hipStream_t s) {
    if (db && p.nnzb > 0) {
        const int gb = ceil_div(p.nnzb, kBlock);
        if (f64)
            hipLaunchKernelGGL(k_grad_b<double>, dim3(gb), dim3(kBlock), 0, s, p,
                               (const double *)av, cri, (const double *)gv, (double *)db, err);
        else
            hipLaunchKernelGGL(k_grad_b<float>, dim3(gb), dim3(kBlock), 0, s, p,
                               (const float *)av, cri, (const float *)gv, (float *)db, err);
    }
    if (da && p.nnza > 0) {
        const int ga = ceil_div(p.nnza, kBlock);
        if (f64)
            hipLaunchKernelGGL(k_grad_a<double>, dim3(ga), dim3(kBlock), 0, s, p,
                               (const double *)bv, cri, (const double *)gv, (double *)da, rowptr,
                               colj, pos, err);
        else
            hipLaunchKernelGGL(k_grad_a<float>, dim3(ga), dim3(kBlock), 0, s, p,
                               (const float *)bv, cri, (const float *)gv, (float *)da, rowptr,
                               colj, pos, err);
    }
    return hipGetLastError();
}

}  // namespace spg
