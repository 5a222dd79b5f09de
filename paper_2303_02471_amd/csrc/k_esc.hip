// Wavefront sort-merge accumulator for the lightest columns: expand, sort,
// compress (ESC, Section 4), one 64-lane wavefront per group of columns.
//
// Sub-bin i holds the columns of at most S = 4 << i products; a group is
// 64 >> i of them and every column owns an aligned segment of S of the
// wavefront's 256 key positions (position s = 64 r + lane for register r).
// The wavefront
//   1. reads the rows of each column's products from the product space (the
//      order the sequential SPA of Algorithm 1 meets them) into its segment as
//      keys (row, e), e the product's position in the column; the rest of the
//      segment is padding that sorts last;
//   2. sorts every segment with the first log2(S) stages of a bitonic network
//      (the last stage ascending everywhere), lane exchanges through DPP,
//      ds_swizzle and ds_bpermute, register exchanges for distances of 64 and
//      more -- a column of at most 4 products takes 3 stages, not the 36 of a
//      full 256-key sort;
//   3. compresses: every run of equal rows is one output entry; its index
//      among the column's runs is its rank (rows come out ascending), and the
//      position of a key inside its run is the occurrence index k of that
//      product among the products Algorithm 1 adds into the entry.
// It writes every column's count and every product's destination: the rank,
// marked for all but the first product of a run, whose k and index among the
// column's later products are stored at the product's position.
//
// Keys are 32-bit when every row index is below 2^24 - 1, else 64-bit.
#include "devutil.h"

namespace spg {

template <typename K>
struct EscSmem {
    long long cbase[64];  // first product of each column of the group
    int op[64];           // products of each column
    int nnz[64];          // entries of each column
    K sk[kEscMaxProducts];     // sorted keys
    int rh[kEscMaxProducts];   // position of each run head, by segment start + run
};

__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int J>
__device__ __forceinline__ unsigned xchg(unsigned v) {
    return (unsigned)shfl_xor_c<J>((int)v);
}
template <int J>
__device__ __forceinline__ unsigned long long xchg(unsigned long long v) {
    return shfl_xor_c64<J>(v);
}

// compare-exchange across lanes at distance J (< 64), every register row;
// position s keeps the smaller key when (ascending) == (s is the lower one)
template <typename K, int J, int S>
__device__ __forceinline__ void esc_lane_step(K (&key)[4], int k, int lane) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int s = r * 64 + lane;
        const K o = xchg<J>(key[r]);
        const bool asc = k == S || (s & k) == 0;
        const bool take_min = asc == ((lane & J) == 0);
        const K mn = key[r] < o ? key[r] : o;
        const K mx = key[r] < o ? o : key[r];
        key[r] = take_min ? mn : mx;
    }
}

// compare-exchange between register rows at distance j >= 64
template <typename K, int S>
__device__ __forceinline__ void esc_reg_step(K (&key)[4], int k, int j, int lane) {
    const int jr = j >> 6;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int rp = r ^ jr;
        if (rp > r) {
            const int s = r * 64 + lane;
            const bool asc = k == S || (s & k) == 0;
            const K x = key[r], y = key[rp];
            const bool sw = asc ? (x > y) : (x < y);
            key[r] = sw ? y : x;
            key[rp] = sw ? x : y;
        }
    }
}

// every aligned segment of S = 1 << LS positions sorted ascending
template <typename K, int LS>
__device__ __forceinline__ void seg_sort(K (&key)[4], int lane) {
    constexpr int S = 1 << LS;
#pragma unroll
    for (int k = 2; k <= S; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            if (j >= 64) {
                esc_reg_step<K, S>(key, k, j, lane);
            } else {
                switch (j) {
                    case 32: esc_lane_step<K, 32, S>(key, k, lane); break;
                    case 16: esc_lane_step<K, 16, S>(key, k, lane); break;
                    case 8: esc_lane_step<K, 8, S>(key, k, lane); break;
                    case 4: esc_lane_step<K, 4, S>(key, k, lane); break;
                    case 2: esc_lane_step<K, 2, S>(key, k, lane); break;
                    default: esc_lane_step<K, 1, S>(key, k, lane); break;
                }
            }
        }
    }
}

template <typename K, int LS>
__device__ __forceinline__ void esc_group(const KArgs &a, EscSmem<K> &S, int first, int ncols,
                                          int lane, int &kmax) {
    constexpr int SEG = 1 << LS;
    constexpr K KMAX = (K)~(K)0;
    // ---- the group's columns, one per lane
    int g = 0;
    if (lane < ncols) {
        g = a.binlist[first + lane].x;
        const int op = a.op[g];
        S.op[lane] = op > SEG ? -1 : op;  // more than planned: cannot happen for unchanged inputs
        S.cbase[lane] = a.colprod[g];
    }
    wave_sync_lds();
    // ---- keys (row, e) in each column's segment
    K key[4];
    bool bad = false;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int s = r * 64 + lane, cc = s >> LS, i = s & (SEG - 1);
        key[r] = KMAX;
        if (cc < ncols) {
            const int op = S.op[cc];
            bad |= op < 0;
            if (i < op) key[r] = ((K)(unsigned)a.prow[S.cbase[cc] + i] << 8) | (K)i;
        }
    }
    if (bad) atomicOr(&a.hdr->err, ERR_GROUP);
    seg_sort<K, LS>(key, lane);
#pragma unroll
    for (int r = 0; r < 4; ++r) S.sk[r * 64 + lane] = key[r];
    wave_sync_lds();
    // ---- runs: heads, run index inside the column
    bool head[4];
    unsigned long long hm[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int s = r * 64 + lane;
        head[r] = key[r] != KMAX && ((s & (SEG - 1)) == 0 || (S.sk[s - 1] >> 8) != (key[r] >> 8));
        hm[r] = ballot(head[r]);
    }
    const unsigned long long le = mask_lt() | (1ull << lane);
    int run[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        int c;
        if (SEG <= 64) {
            // the segment lies inside register row r
            const int ls = lane & ~(SEG - 1);
            const unsigned long long seg = SEG == 64 ? ~0ull : (((1ull << SEG) - 1ull) << ls);
            c = popc64(hm[r] & le & seg);
        } else {
            // the segment starts at lane 0 of row r0 and spans SEG / 64 rows
            constexpr int RS = SEG / 64;
            const int r0 = r & ~(RS - 1);
            c = popc64(hm[r] & le);
#pragma unroll
            for (int q = 0; q < 4; ++q)
                if (q >= r0 && q < r) c += popc64(hm[q]);
        }
        run[r] = c - 1;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int s = r * 64 + lane, ss = s & ~(SEG - 1);
        if (head[r]) S.rh[ss + run[r]] = s;
        // the last key of a column holds its entry count
        const int cc = s >> LS;
        if (key[r] != KMAX && (s - ss) == S.op[cc] - 1) S.nnz[cc] = run[r] + 1;
    }
    wave_sync_lds();
    if (lane < ncols) a.gnnz[g] = S.op[lane] > 0 ? S.nnz[lane] : 0;
    // ---- destinations
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        if (key[r] == KMAX) continue;
        const int s = r * 64 + lane, ss = s & ~(SEG - 1), cc = s >> LS;
        const int e = (int)(key[r] & (K)255);
        const int k = s - S.rh[ss + run[r]];
        const long long pe = S.cbase[cc] + e;
        if (k == 0) {
            a.dst[pe] = (uint32_t)run[r];
        } else {
            // later keys before this one inside the column
            a.dst[pe] = kDstLater | (uint32_t)run[r];
            a.lk[pe] = k;
            a.lr[pe] = (s - ss) - run[r] - 1;
            kmax = max(kmax, k);
        }
    }
    wave_sync_lds();  // the LDS of this group is read before the next group writes it
}

// one launch per sub-bin: sub-bin LS - 2 holds columns of at most 1 << LS
// products, 64 >> (LS - 2) of them per wavefront group
template <typename K, int LS>
__global__ __launch_bounds__(kBlock) void k_esc(KArgs a) {
    __shared__ EscSmem<K> smem[kBlock / 64];
    if (a.hdr->err) return;
    const int lane = lane_id();
    EscSmem<K> &S = smem[threadIdx.x >> 6];
    constexpr int sb = LS - 2, G = 64 >> sb;
    int start = 0;
    for (int b = 0; b < BIN_ESC0 + sb; ++b) start += a.hdr->bin_count[b];
    const int cnt = a.hdr->bin_count[BIN_ESC0 + sb];
    const int ngroups = ceil_div(cnt, G);
    const int wstride = gridDim.x * (kBlock / 64);
    int kmax = 0;
    for (int gi = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6); gi < ngroups; gi += wstride)
        esc_group<K, LS>(a, S, start + gi * G, min(G, cnt - gi * G), lane, kmax);
    // the largest occurrence index (a device atomic only when it raises the
    // value already there)
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1)
        kmax = max(kmax, __builtin_amdgcn_ds_bpermute((lane ^ d) << 2, kmax));
    if (lane == 0 && kmax > __atomic_load_n(&a.hdr->later_maxk, __ATOMIC_RELAXED))
        atomicMax(&a.hdr->later_maxk, kmax);
}

// All sub-bins in one launch, the largest first: position j of the launch
// order is sub-bin r.sub[j], with the workgroups [r.first[j], r.first[j + 1]).
struct EscRanges {
    int first[kEscBins + 1];
    int sub[kEscBins];
};

template <typename K, int LS>
__device__ __forceinline__ void esc_sub(const KArgs &a, EscSmem<K> &S, int blk, int nblk,
                                        int lane, int &kmax) {
    constexpr int sb = LS - 2, G = 64 >> sb;
    int start = 0;
    for (int b = 0; b < BIN_ESC0 + sb; ++b) start += a.hdr->bin_count[b];
    const int cnt = a.hdr->bin_count[BIN_ESC0 + sb];
    const int ngroups = ceil_div(cnt, G);
    const int wstride = nblk * (kBlock / 64);
    for (int gi = blk * (kBlock / 64) + (threadIdx.x >> 6); gi < ngroups; gi += wstride)
        esc_group<K, LS>(a, S, start + gi * G, min(G, cnt - gi * G), lane, kmax);
}

template <typename K>
__global__ __launch_bounds__(kBlock) void k_esc_all(KArgs a, EscRanges r) {
    __shared__ EscSmem<K> smem[kBlock / 64];
    if (a.hdr->err) return;
    const int lane = lane_id();
    EscSmem<K> &S = smem[threadIdx.x >> 6];
    int j = 0;
    while (j + 1 < kEscBins && (int)blockIdx.x >= r.first[j + 1]) ++j;
    const int blk = (int)blockIdx.x - r.first[j], nblk = r.first[j + 1] - r.first[j];
    int kmax = 0;
    switch (r.sub[j]) {
        case 0: esc_sub<K, 2>(a, S, blk, nblk, lane, kmax); break;
        case 1: esc_sub<K, 3>(a, S, blk, nblk, lane, kmax); break;
        case 2: esc_sub<K, 4>(a, S, blk, nblk, lane, kmax); break;
        case 3: esc_sub<K, 5>(a, S, blk, nblk, lane, kmax); break;
        case 4: esc_sub<K, 6>(a, S, blk, nblk, lane, kmax); break;
        case 5: esc_sub<K, 7>(a, S, blk, nblk, lane, kmax); break;
        default: esc_sub<K, 8>(a, S, blk, nblk, lane, kmax); break;
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1)
        kmax = max(kmax, __builtin_amdgcn_ds_bpermute((lane ^ d) << 2, kmax));
    if (lane == 0 && kmax > __atomic_load_n(&a.hdr->later_maxk, __ATOMIC_RELAXED))
        atomicMax(&a.hdr->later_maxk, kmax);
}

// groups[i]: wavefront groups of sub-bin i (0 skips it)
hipError_t launch_esc_all(const KArgs &a, bool wide, const int *groups, hipStream_t s) {
    EscRanges r{};
    int tot = 0;
    for (int j = 0; j < kEscBins; ++j) {
        const int i = kEscBins - 1 - j;
        r.sub[j] = i;
        r.first[j] = tot;
        tot += ceil_div(groups[i], kBlock / 64);
    }
    r.first[kEscBins] = tot;
    if (tot == 0) return hipSuccess;
    if (wide) hipLaunchKernelGGL((k_esc_all<unsigned long long>), dim3(tot), dim3(kBlock), 0, s, a, r);
    else hipLaunchKernelGGL((k_esc_all<unsigned>), dim3(tot), dim3(kBlock), 0, s, a, r);
    return hipGetLastError();
}

hipError_t launch_esc(const KArgs &a, bool wide, int sub, int groups, hipStream_t s) {
    if (groups <= 0) return hipSuccess;
    const dim3 grid(ceil_div(groups, kBlock / 64));
#define SPG_ESC(K)                                                                       \
    switch (sub) {                                                                       \
        case 0: hipLaunchKernelGGL((k_esc<K, 2>), grid, dim3(kBlock), 0, s, a); break;   \
        case 1: hipLaunchKernelGGL((k_esc<K, 3>), grid, dim3(kBlock), 0, s, a); break;   \
        case 2: hipLaunchKernelGGL((k_esc<K, 4>), grid, dim3(kBlock), 0, s, a); break;   \
        case 3: hipLaunchKernelGGL((k_esc<K, 5>), grid, dim3(kBlock), 0, s, a); break;   \
        case 4: hipLaunchKernelGGL((k_esc<K, 6>), grid, dim3(kBlock), 0, s, a); break;   \
        case 5: hipLaunchKernelGGL((k_esc<K, 7>), grid, dim3(kBlock), 0, s, a); break;   \
        default: hipLaunchKernelGGL((k_esc<K, 8>), grid, dim3(kBlock), 0, s, a); break;  \
    }
    if (wide) SPG_ESC(unsigned long long)
    else SPG_ESC(unsigned)
#undef SPG_ESC
    return hipGetLastError();
}

}  // namespace spg
