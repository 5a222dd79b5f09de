// Block sort accumulator for medium columns (more products than the
// wavefront sort-merge takes, at most 4096): the expand-sort-compress
// scheme of Section 4 at workgroup scale, one workgroup per column.
//
// The workgroup reads the rows of the column's products from the product
// space (Algorithm 1 order), forms the keys (row, e) with e the position in
// that order, and sorts them with a bitonic network: exchanges at distance
// below 64 move through DPP / ds_swizzle / ds_bpermute, distances 64..128
// between the four registers a lane holds, and larger distances through LDS.
// Before the network, the workgroup tries a bucket sort, which does far less
// work when the rows are spread out: the span [lo, hi] of the column's rows is
// cut into one bucket per thread by a monotone map, keys are counted and
// scattered to their buckets in LDS, and every thread sorts its own bucket by
// insertion. Buckets are in row order and every key is unique, so the result
// is the same ascending order the network gives. If any bucket would exceed
// kBucketCap keys (clustered or repeated rows), the column takes the network.
//
// Every run of equal rows is one output entry; its rank is the run index and
// the position of a key inside its run is the occurrence index k of that
// product. Every product gets the rank as its destination, marked for all but
// the first of a run, whose occurrence index k and index among the column's
// later products are stored at the product's position.
//
// Keys are 32-bit when the rows fit in 20 bits (row << 12 | e), else 64-bit.
#include "devutil.h"

namespace spg {

template <typename K>
struct KeyMax;
template <>
struct KeyMax<unsigned> {
    static constexpr unsigned v = ~0u;
};
template <>
struct KeyMax<unsigned long long> {
    static constexpr unsigned long long v = ~0ull;
};

template <int J>
__device__ __forceinline__ unsigned xshfl(unsigned v) {
    return (unsigned)shfl_xor_c<J>((int)v);
}
template <int J>
__device__ __forceinline__ unsigned long long xshfl(unsigned long long v) {
    return shfl_xor_c64<J>(v);
}

// key[r] of lane l sits at position sb + 64 r + l. A position takes the
// smaller key of its pair when (ascending block) == (lower element).
template <typename K, int J>
__device__ __forceinline__ void lane_step(K (&key)[4], int k, int sb, int lane) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int s = sb + r * 64 + lane;
        const K o = xshfl<J>(key[r]);
        const bool take_min = ((s & k) == 0) == ((lane & J) == 0);
        const K mn = key[r] < o ? key[r] : o;
        const K mx = key[r] < o ? o : key[r];
        key[r] = take_min ? mn : mx;
    }
}

template <typename K>
__device__ __forceinline__ void reg_step(K (&key)[4], int k, int j, int sb, int lane) {
    const int jr = j >> 6;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int rp = r ^ jr;
        if (rp > r) {
            const int s = sb + r * 64 + lane;
            const bool asc = (s & k) == 0;
            const K x = key[r], y = key[rp];
            const bool sw = asc ? (x > y) : (x < y);
            key[r] = sw ? y : x;
            key[rp] = sw ? x : y;
        }
    }
}

// partner in another wavefront's 256 positions: exchange through LDS
template <typename K>
__device__ __forceinline__ void lds_step(K (&key)[4], K *buf, int k, int j, int sb, int lane) {
#pragma unroll
    for (int r = 0; r < 4; ++r) buf[sb + r * 64 + lane] = key[r];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int s = sb + r * 64 + lane;
        const K o = buf[s ^ j];
        const bool take_min = ((s & k) == 0) == ((s & j) == 0);
        const K mn = key[r] < o ? key[r] : o;
        const K mx = key[r] < o ? o : key[r];
        key[r] = take_min ? mn : mx;
    }
    __syncthreads();
}

// ascending sort of the workgroup's N = 4 * threads keys
template <typename K, int N>
__device__ __forceinline__ void block_sort(K (&key)[4], K *buf) {
    const int lane = lane_id(), sb = (threadIdx.x >> 6) * 256;
#pragma unroll
    for (int k = 2; k <= N; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            if (j >= 256) {
                lds_step(key, buf, k, j, sb, lane);
            } else if (j >= 64) {
                reg_step(key, k, j, sb, lane);
            } else {
                switch (j) {
                    case 32: lane_step<K, 32>(key, k, sb, lane); break;
                    case 16: lane_step<K, 16>(key, k, sb, lane); break;
                    case 8: lane_step<K, 8>(key, k, sb, lane); break;
                    case 4: lane_step<K, 4>(key, k, sb, lane); break;
                    case 2: lane_step<K, 2>(key, k, sb, lane); break;
                    default: lane_step<K, 1>(key, k, sb, lane); break;
                }
            }
        }
    }
}

constexpr int kBucketCap = 24;  // most keys a bucket of the bucket sort takes

// smallest and largest of lo / hi over the workgroup (red: 2 * NW ints);
// ends with a barrier
template <int NW>
__device__ __forceinline__ void wg_minmax(int &lo, int &hi, int *red) {
    lo = min(lo, shfl_xor_c<32>(lo));
    hi = max(hi, shfl_xor_c<32>(hi));
    lo = min(lo, shfl_xor_c<16>(lo));
    hi = max(hi, shfl_xor_c<16>(hi));
    lo = min(lo, shfl_xor_c<8>(lo));
    hi = max(hi, shfl_xor_c<8>(hi));
    lo = min(lo, shfl_xor_c<4>(lo));
    hi = max(hi, shfl_xor_c<4>(hi));
    lo = min(lo, shfl_xor_c<2>(lo));
    hi = max(hi, shfl_xor_c<2>(hi));
    lo = min(lo, shfl_xor_c<1>(lo));
    hi = max(hi, shfl_xor_c<1>(hi));
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[w] = lo;
        red[NW + w] = hi;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        lo = min(lo, red[i]);
        hi = max(hi, red[NW + i]);
    }
}

template <typename K, int T>
__global__ __launch_bounds__(T, 8) void k_bsort(KArgs a, int bin) {
    constexpr int N = 4 * T, NW = T / 64;
    constexpr int EB = 12;  // bits of the product position (N <= 4096)
    constexpr K KMAX = KeyMax<K>::v;
    static_assert(N <= (1 << EB), "positions must fit the key");
    __shared__ K buf[N];     // exchanges, then the sorted keys
    __shared__ int rh[N];    // bucket counts and starts, then the sorted position of every run head
    __shared__ int wcnt[NW + 1];
    __shared__ int red[2 * NW];
    __shared__ int s_kmax;
    if (__syncthreads_or(__atomic_load_n(&a.hdr->err, __ATOMIC_RELAXED) != 0))
        return;  // every thread takes the same branch
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, sb = wave * 256;
    int start = 0;
    for (int b = 0; b < bin; ++b) start += a.hdr->bin_count[b];
    const int ncols = a.hdr->bin_count[bin];
    for (int ci = blockIdx.x; ci < ncols; ci += gridDim.x) {
        const int g = a.binlist[start + ci].x;
        const int op = a.op[g];
        const long long pbase = a.colprod[g];
        if (op > N) {  // cannot happen: the classification bounds the bin
            if (tid == 0) atomicOr(&a.hdr->err, ERR_GROUP);
            continue;
        }
        int row[4];
        int lo = 0x7fffffff, hi = -1;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int s = sb + r * 64 + lane;
            row[r] = s < op ? a.prow[pbase + s] : -1;
            if (row[r] >= 0) {
                lo = min(lo, row[r]);
                hi = max(hi, row[r]);
            }
        }
        rh[tid] = 0;
        wg_minmax<NW>(lo, hi, red);  // its barrier also orders the zeroing
        // bucket of a row: monotone in the row, so buckets are in row order
        const float scale = (float)T / (float)(hi - lo + 1);
        int bk[4], slot[4];
        bool ovf = false;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            bk[r] = 0;
            slot[r] = 0;
            if (row[r] >= 0) {
                bk[r] = min((int)((float)(row[r] - lo) * scale), T - 1);
                slot[r] = atomicAdd(&rh[bk[r]], 1);
                ovf |= slot[r] >= kBucketCap;
            }
        }
        K key[4];
        if (!__syncthreads_or(ovf)) {
            const int cnt = rh[tid];
            int tot;
            const int st = wg_excl_scan<T>(cnt, wcnt, tot);
            rh[tid] = st;
            __syncthreads();
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int s = sb + r * 64 + lane;
                if (row[r] >= 0) buf[rh[bk[r]] + slot[r]] = ((K)row[r] << EB) | (K)s;
            }
            __syncthreads();
            // insertion sort of this thread's bucket (keys are unique)
            for (int i = st + 1; i < st + cnt; ++i) {
                const K x = buf[i];
                int j = i - 1;
                K y = buf[j];
                while (y > x) {
                    buf[j + 1] = y;
                    if (--j < st) break;
                    y = buf[j];
                }
                buf[j + 1] = x;
            }
            __syncthreads();
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int s = sb + r * 64 + lane;
                key[r] = s < op ? buf[s] : KMAX;
            }
        } else {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int s = sb + r * 64 + lane;
                key[r] = row[r] >= 0 ? (((K)row[r] << EB) | (K)s) : KMAX;
            }
            block_sort<K, N>(key, buf);
#pragma unroll
            for (int r = 0; r < 4; ++r) buf[sb + r * 64 + lane] = key[r];
            __syncthreads();
        }

        // run heads and run indices (position order: wavefront, register, lane)
        bool head[4];
        int run[4];
        int before = 0;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int s = sb + r * 64 + lane;
            head[r] = key[r] != KMAX && (s == 0 || (buf[s - 1] >> EB) != (key[r] >> EB));
            const unsigned long long m = ballot(head[r]);
            run[r] = before + popc64(m & mask_lt()) - (head[r] ? 0 : 1);
            before += popc64(m);
        }
        if (lane == 0) wcnt[wave] = before;
        __syncthreads();
        if (tid == 0) {
            int tot = 0;
            for (int w = 0; w < NW; ++w) {
                const int x = wcnt[w];
                wcnt[w] = tot;
                tot += x;
            }
            wcnt[NW] = tot;
            s_kmax = 0;
            a.gnnz[g] = tot;
        }
        __syncthreads();
        const int woff = wcnt[wave];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            run[r] += woff;
            if (head[r]) rh[run[r]] = sb + r * 64 + lane;
        }
        __syncthreads();
        int kloc = 0;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            if (key[r] == KMAX) continue;
            const int s = sb + r * 64 + lane;
            const int e = (int)(key[r] & (K)((1 << EB) - 1));
            const int k = s - rh[run[r]];
            if (k == 0) {
                a.dst[pbase + e] = (uint32_t)run[r];
            } else {
                // index among the column's later products: the later keys
                // before this one in sorted order
                a.dst[pbase + e] = kDstLater | (uint32_t)run[r];
                a.lk[pbase + e] = k;
                a.lr[pbase + e] = s - run[r] - 1;
                kloc = max(kloc, k);
            }
        }
        if (kloc) atomicMax(&s_kmax, kloc);
        __syncthreads();
        if (tid == 0 && s_kmax > __atomic_load_n(&a.hdr->later_maxk, __ATOMIC_RELAXED))
            atomicMax(&a.hdr->later_maxk, s_kmax);
    }
}

// ---------------------------------------------------------------- windowed sort
// Columns of more than kSortMax products: the column's rows [lo, hi] are cut
// into W windows of equal row span, W planned for about 3/4 of a sort each;
// one workgroup takes the windows in row order, sorting the products of each
// (in product order) like k_bsort and carrying the ranks and the later-product
// indices of the earlier windows. A window holding more than kSortMax
// products is split in halves; a window of a single row (any number of
// products: one entry) needs no sort, its products take their occurrence
// indices in product order.
constexpr int kWinDepth = 48;

template <typename K>
__global__ __launch_bounds__(1024) void k_wsort(KArgs a) {
    constexpr int T = 1024, N = 4 * T, NW = T / 64;
    constexpr int EB = 12;  // bits of a window position (N <= 4096)
    constexpr K KMAX = KeyMax<K>::v;
    static_assert(N <= (1 << EB), "positions must fit the key");
    __shared__ K buf[N];     // keys, exchanges, then the sorted keys
    __shared__ int rh[N];    // sorted position of every run head
    __shared__ int emap[N];  // product position of every window position
    __shared__ int bfill[T];        // bucket fill counters of the bucket sort
    __shared__ int wcnt[NW + 1];
    __shared__ int scan_tmp[NW + 1];
    __shared__ int stk_lo[kWinDepth], stk_hi[kWinDepth];
    __shared__ int s_min, s_max, s_kmax;
    if (__syncthreads_or(__atomic_load_n(&a.hdr->err, __ATOMIC_RELAXED) != 0))
        return;  // every thread takes the same branch
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, sb = wave * 256;
    int first = 0;
    for (int b = 0; b < BIN_WSORT; ++b) first += a.hdr->bin_count[b];
    const int n = a.hdr->bin_count[BIN_WSORT];
    if (tid == 0) s_kmax = 0;
    int kmax = 0;
    bool abort = false;  // workgroup-uniform
    for (int li = blockIdx.x; li < n && !abort; li += gridDim.x) {
        const int g = a.binlist[first + li].x;
        const int op = a.op[g];
        const long long pbase = a.colprod[g];
        const int *__restrict__ prow = a.prow + pbase;
        uint32_t *__restrict__ dstp = a.dst + pbase;
        // row span of the column (the window passes re-read the rows, which
        // stay in L2)
        if (tid == 0) {
            s_min = 0x7fffffff;
            s_max = -1;
        }
        int mn = 0x7fffffff, mx = -1;
        for (int e = tid; e < op; e += 4 * T) {
            int r[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) r[u] = e + u * T < op ? prow[e + u * T] : -1;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (r[u] < 0) continue;
                mn = min(mn, r[u]);
                mx = max(mx, r[u]);
            }
        }
        auto row_at = [&](int e) { return prow[e]; };
        __syncthreads();
        {
#pragma unroll
            for (int d = 32; d >= 1; d >>= 1) {
                mn = min(mn, __builtin_amdgcn_ds_bpermute((lane ^ d) << 2, mn));
                mx = max(mx, __builtin_amdgcn_ds_bpermute((lane ^ d) << 2, mx));
            }
            if (lane == 0) {
                atomicMin(&s_min, mn);
                atomicMax(&s_max, mx);
            }
        }
        __syncthreads();
        const int lo = s_min, span = s_max + 1 - s_min;
        const int q = ceil_div(op, T);
        const int e0 = min(op, tid * q), e1 = min(op, e0 + q);
        // windows planned for about 0.9 of a sort (a window above N splits)
        int W = ceil_div(op, 9 * N / 10);
        if (W > span) W = span;
        int total = 0, ltotal = 0;
        for (int w = 0; w < W && !abort; ++w) {
            if (tid == 0) {
                stk_lo[0] = lo + (int)((long long)w * span / W);
                stk_hi[0] = lo + (int)((long long)(w + 1) * span / W);
            }
            int sp = 1;
            __syncthreads();
            while (sp > 0) {
                --sp;
                const int x = stk_lo[sp], y = stk_hi[sp];
                // the window's products, numbered in product order, and their
                // bucket counts (one bucket per thread over the window's rows)
                const float scale = (float)T / (float)(y - x);
                rh[tid] = 0;
                bfill[tid] = 0;
                __syncthreads();
                int c = 0;
                bool ovf = false;
                for (int e = e0; e < e1; ++e) {
                    const int r = row_at(e);
                    if (r >= x && r < y) {
                        ++c;
                        const int b = min((int)((float)(r - x) * scale), T - 1);
                        ovf |= atomicAdd(&rh[b], 1) >= kBucketCap;
                    }
                }
                ovf = __syncthreads_or(ovf);
                int cnt;
                const int off = wg_excl_scan<T>(c, scan_tmp, cnt);
                if (cnt > N && y - x > 1) {
                    // split; the left half is taken first
                    if (sp + 2 > kWinDepth) {  // cannot happen: the span halves each time
                        abort = true;
                        break;
                    }
                    const int mid = x + (y - x) / 2;
                    if (tid == 0) {
                        stk_lo[sp] = mid; stk_hi[sp] = y;
                        stk_lo[sp + 1] = x; stk_hi[sp + 1] = mid;
                    }
                    sp += 2;
                    __syncthreads();
                    continue;
                }
                if (cnt > N) {
                    // one row: one entry; occurrence indices in product order
                    int k = off;
                    for (int e = e0; e < e1; ++e) {
                        const int r = row_at(e);
                        if (r < x || r >= y) continue;
                        if (k == 0) {
                            dstp[e] = (uint32_t)total;
                        } else {
                            dstp[e] = kDstLater | (uint32_t)total;
                            a.lk[pbase + e] = k;
                            a.lr[pbase + e] = ltotal + k - 1;
                            kmax = max(kmax, k);
                        }
                        ++k;
                    }
                    total += 1;
                    ltotal += cnt - 1;
                    __syncthreads();
                    continue;
                }
                // keys (row, window position): scattered to their buckets and
                // sorted there, or (a bucket too full) sorted by the network
                K key[4];
                if (!ovf) {
                    const int bc = rh[tid];
                    int bt;
                    const int bst = wg_excl_scan<T>(bc, scan_tmp, bt);
                    rh[tid] = bst;
                    __syncthreads();
                    int i = off;
                    for (int e = e0; e < e1; ++e) {
                        const int r = row_at(e);
                        if (r < x || r >= y) continue;
                        emap[i] = e;
                        const int b = min((int)((float)(r - x) * scale), T - 1);
                        buf[rh[b] + atomicAdd(&bfill[b], 1)] = ((K)r << EB) | (K)i;
                        ++i;
                    }
                    __syncthreads();
                    for (int u = bst + 1; u < bst + bc; ++u) {
                        const K v = buf[u];
                        int j = u - 1;
                        K y2 = buf[j];
                        while (y2 > v) {
                            buf[j + 1] = y2;
                            if (--j < bst) break;
                            y2 = buf[j];
                        }
                        buf[j + 1] = v;
                    }
                    __syncthreads();
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int s = sb + r * 64 + lane;
                        key[r] = s < cnt ? buf[s] : KMAX;
                    }
                } else {
                    int i = off;
                    for (int e = e0; e < e1; ++e) {
                        const int r = row_at(e);
                        if (r < x || r >= y) continue;
                        emap[i] = e;
                        buf[i] = ((K)r << EB) | (K)i;
                        ++i;
                    }
                    __syncthreads();
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int s = sb + r * 64 + lane;
                        key[r] = s < cnt ? buf[s] : KMAX;
                    }
                    __syncthreads();
                    block_sort<K, N>(key, buf);
#pragma unroll
                    for (int r = 0; r < 4; ++r) buf[sb + r * 64 + lane] = key[r];
                    __syncthreads();
                }
                // run heads and run indices (position order: wavefront, register, lane)
                bool head[4];
                int run[4];
                int before = 0;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int s = sb + r * 64 + lane;
                    head[r] = key[r] != KMAX && (s == 0 || (buf[s - 1] >> EB) != (key[r] >> EB));
                    const unsigned long long m = ballot(head[r]);
                    run[r] = before + popc64(m & mask_lt()) - (head[r] ? 0 : 1);
                    before += popc64(m);
                }
                if (lane == 0) wcnt[wave] = before;
                __syncthreads();
                if (tid == 0) {
                    int tot = 0;
                    for (int v = 0; v < NW; ++v) {
                        const int t = wcnt[v];
                        wcnt[v] = tot;
                        tot += t;
                    }
                    wcnt[NW] = tot;
                }
                __syncthreads();
                const int woff = wcnt[wave], runs = wcnt[NW];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    run[r] += woff;
                    if (head[r]) rh[run[r]] = sb + r * 64 + lane;
                }
                __syncthreads();
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    if (key[r] == KMAX) continue;
                    const int s = sb + r * 64 + lane;
                    const int e = emap[(int)(key[r] & (K)((1 << EB) - 1))];
                    const int k = s - rh[run[r]];
                    const int rank = total + run[r];
                    if (k == 0) {
                        dstp[e] = (uint32_t)rank;
                    } else {
                        dstp[e] = kDstLater | (uint32_t)rank;
                        a.lk[pbase + e] = k;
                        a.lr[pbase + e] = ltotal + (s - run[r] - 1);
                        kmax = max(kmax, k);
                    }
                }
                total += runs;
                ltotal += cnt - runs;
                __syncthreads();
            }
        }
        if (tid == 0) a.gnnz[g] = total;
    }
    if (abort && tid == 0) atomicOr(&a.hdr->err, ERR_GROUP);
    if (kmax) atomicMax(&s_kmax, kmax);
    __syncthreads();
    if (tid == 0 && s_kmax > __atomic_load_n(&a.hdr->later_maxk, __ATOMIC_RELAXED))
        atomicMax(&a.hdr->later_maxk, s_kmax);
}

hipError_t launch_wsort(const KArgs &a, bool wide, int grid, hipStream_t s) {
    if (grid <= 0) return hipSuccess;
    if (wide) hipLaunchKernelGGL((k_wsort<unsigned long long>), dim3(grid), dim3(1024), 0, s, a);
    else hipLaunchKernelGGL((k_wsort<unsigned>), dim3(grid), dim3(1024), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_sort(const KArgs &a, int cls, bool wide, int grid, hipStream_t s) {
    if (grid <= 0) return hipSuccess;
    const int bin = BIN_SORT0 + cls;  // columns of at most 512 << cls products
#define SPG_SORT(K, T) hipLaunchKernelGGL((k_bsort<K, T>), dim3(grid), dim3(T), 0, s, a, bin)
    if (wide) {
        switch (cls) {
            case 0: SPG_SORT(unsigned long long, 128); break;
            case 1: SPG_SORT(unsigned long long, 256); break;
            case 2: SPG_SORT(unsigned long long, 512); break;
            default: SPG_SORT(unsigned long long, 1024); break;
        }
    } else {
        switch (cls) {
            case 0: SPG_SORT(unsigned, 128); break;
            case 1: SPG_SORT(unsigned, 256); break;
            case 2: SPG_SORT(unsigned, 512); break;
            default: SPG_SORT(unsigned, 1024); break;
        }
    }
#undef SPG_SORT
    return hipGetLastError();
}

}  // namespace spg
