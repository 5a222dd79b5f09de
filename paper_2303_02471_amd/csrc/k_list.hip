// Product lists of the dense and hash columns.
//
// For every such column the products of Gustavson's column method (Section
// 2.1) are expanded once, in the order Algorithm 1 meets them (stored B
// entries in storage order, then the rows of the selected A column in storage
// order), and written as (row) and (A entry q, B entry p) into the column's
// list segment. Columns processed in several row windows get their segment
// partitioned by window with a stable counting sort, so that each window's
// products stay in Algorithm 1 order. The accumulators then stream their
// window's contiguous slice; the numeric phase only gathers A(q) and B(p).
#include "devutil.h"

namespace spg {

constexpr int kLT = 256;  // threads per list workgroup

// op of every list column, in bin-list order (input of the offset scan)
__global__ __launch_bounds__(kBlock) void k_list_ops(KArgs a, int first, int n, int32_t *out) {
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) out[i] = a.op[a.binlist[first + i].x];
}

struct ListSmem {
    int s_acp[kLT];
    int s_eoff[kLT];
    int scan_tmp[kLT / 64 + 1];
    int cnt[kMaxWindows];   // products per window, then the running fill position
    int s_err;
};

// Walks the products of one column in Algorithm 1 order and calls
// f(e, row, q, p) for each; all threads of the workgroup must call it.
template <typename F>
__device__ __forceinline__ void for_each_product(const Prob &d, const int2 *E, int bs, int be,
                                                 ListSmem &S, F &&f) {
    const int tid = threadIdx.x;
    int ebase = 0;
    for (int bw = bs; bw < be; bw += kLT) {
        const int t = bw + tid;
        int z = 0, acp = 0;
        if (t < be) {
            const int2 ez = E[t];
            acp = ez.x;
            z = ez.y;
        }
        int Ew;
        const int ex = block_excl_scan(z, S.scan_tmp, Ew);
        S.s_acp[tid] = acp;
        S.s_eoff[tid] = ex;
        __syncthreads();
        const int nbw = min(kLT, be - bw);
        for (int e0 = 0; e0 < Ew; e0 += kLT) {
            const int e = e0 + tid;
            int row = -1, q = 0, p = 0;
            if (e < Ew) {
                const int tt = last_le(S.s_eoff, nbw, e);
                q = S.s_acp[tt] + e - S.s_eoff[tt];
                p = bw + tt;
                row = d.ari[q];
                if (row < 0 || row >= d.m) {
                    S.s_err = ERR_CSC;
                    row = 0;
                }
            }
            f(e < Ew, ebase + e, row, q, p);
        }
        ebase += Ew;
        __syncthreads();
    }
}

__global__ __launch_bounds__(kLT) void k_lists(KArgs a, int first, int n) {
    __shared__ ListSmem S;
    if (a.hdr->err) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int li = blockIdx.x; li < n; li += gridDim.x) {
        const int pos = first + li;
        const int4 ent = a.binlist[pos];
        const int g = ent.x, bs = ent.y, be = ent.y + ent.z;
        const int pid = find_prob(a, g);
        const Prob d = get_prob(a, pid);
        const int bw = a.binw[g];
        const int bin = bw & 255;
        const int W = max(bw >> 8, 1);
        const long long base = a.colprod[li];
        const int item0 = bin >= BIN_HASH_S ? a.colitem[pos] : -1;
        const int2 *E = a.E + d.ebase;
        if (tid == 0) S.s_err = 0;
        __syncthreads();
        if (W == 1) {
            for_each_product(d, E, bs, be, S, [&](bool ok, int e, int row, int q, int p) {
                if (ok) {
                    a.lrow[base + e] = row;
                    a.lqp[base + e] = make_int2(q, p);
                }
            });
            if (item0 >= 0 && tid == 0) {
                a.itemstart[item0] = base;
                a.itemlen[item0] = a.op[g];
            }
        } else {
            // pass 1: products per window
            for (int w = tid; w < W; w += kLT) S.cnt[w] = 0;
            __syncthreads();
            for_each_product(d, E, bs, be, S, [&](bool ok, int, int row, int, int) {
                if (ok) atomicAdd(&S.cnt[window_of(row, W, d.m)], 1);
            });
            // window starts (exclusive scan, W <= kMaxWindows entries)
            if (tid == 0) {
                int run = 0;
                for (int w = 0; w < W; ++w) {
                    const int c = S.cnt[w];
                    a.itemstart[item0 + w] = base + run;
                    a.itemlen[item0 + w] = c;
                    S.cnt[w] = run;
                    run += c;
                }
            }
            __syncthreads();
            // pass 2: stable scatter; the waves of a chunk take turns so that
            // positions follow Algorithm 1 order inside every window
            for_each_product(d, E, bs, be, S, [&](bool ok, int, int row, int q, int p) {
                const int w = ok ? window_of(row, W, d.m) : -1;
                int mypos = -1;
                for (int turn = 0; turn < kLT / 64; ++turn) {
                    if (turn == wave) {
                        unsigned long long todo = ballot(ok);
                        while (todo) {
                            const int leader = __builtin_ctzll(todo);
                            const int lw = __builtin_amdgcn_readlane(w, leader);
                            const unsigned long long m = ballot(ok && w == lw);
                            const int before = S.cnt[lw];
                            if (ok && w == lw) mypos = before + popc64(m & mask_lt());
                            if (lane == leader) S.cnt[lw] = before + popc64(m);
                            todo &= ~m;
                        }
                    }
                    __syncthreads();
                }
                if (ok) {
                    a.lrow[base + mypos] = row;
                    a.lqp[base + mypos] = make_int2(q, p);
                }
            });
        }
        __syncthreads();
        if (tid == 0 && S.s_err) atomicOr(&a.hdr->err, S.s_err);
    }
}

hipError_t launch_lists(const KArgs &a, int first, int ncols_list, int32_t *tmp, long long *bsum,
                        int nbsum, hipStream_t s) {
    if (ncols_list <= 0) return hipSuccess;
    // list segment of every column: exclusive scan of Op over the list columns
    hipLaunchKernelGGL(k_list_ops, dim3(ceil_div(ncols_list, kBlock)), dim3(kBlock), 0, s, a,
                       first, ncols_list, tmp);
    hipError_t e = launch_scan_i64(tmp, ncols_list, bsum, nbsum, a.colprod, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_lists, dim3(ncols_list), dim3(kLT), 0, s, a, first, ncols_list);
    return hipGetLastError();
}

}  // namespace spg
