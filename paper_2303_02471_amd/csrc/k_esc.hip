// Wavefront sort-merge accumulator for the lightest columns: expand, sort,
// compress (ESC, Section 4), one 64-lane wavefront per group of columns.
//
// A group holds up to 64 columns whose products and stored B entries each add
// up to at most 256. The wavefront
//   1. reads the rows of the group's products from the product space (each
//      column's products in the order the sequential SPA of Algorithm 1 meets
//      them); e is the position in the group;
//   2. sorts the keys (column, row, e) with a register bitonic network whose
//      lane exchanges use DPP, ds_swizzle and ds_bpermute;
//   3. compresses: every (column, row) run is one output entry; its rank
//      inside the column is its output position (rows come out ascending),
//      and the position of a key inside its run is the occurrence index k of
//      that product among the products Algorithm 1 adds into the entry.
// It counts the runs per column and records the destination of every
// product: the rank of its row, marked for all but the first product of a run,
// whose occurrence index k and index among the column's later products are
// stored at the product's position.
#include "devutil.h"

namespace spg {

struct EscSmem {
    int goff[65];    // first product of each column inside the group
    long long cbase[64];  // first product of each column in the product space
    int cnt[65];     // first run index of each column
    unsigned long long sk[kEscMaxProducts];  // sorted keys
    int rh[kEscMaxProducts];                 // sorted position of every run head
};

__device__ __forceinline__ void wave_sync_lds() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// compare-exchange across lanes at distance J (< 64) for every register row
template <int R, int J>
__device__ __forceinline__ void bitonic_lane_step(unsigned long long (&key)[4], int k, int lane) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int s = r * 64 + lane;
        unsigned long long o = shfl_xor_c64<J>(key[r]);
        const bool asc = (s & k) == 0;
        const bool lower = (lane & J) == 0;
        const unsigned long long mn = key[r] < o ? key[r] : o;
        const unsigned long long mx = key[r] < o ? o : key[r];
        key[r] = (asc == lower) ? mn : mx;
    }
}

// compare-exchange between register rows at distance J >= 64
template <int R>
__device__ __forceinline__ void bitonic_reg_step(unsigned long long (&key)[4], int k, int j,
                                                 int lane) {
    const int jr = j >> 6;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int rp = r ^ jr;
        if (rp > r && rp < R) {
            const int s = r * 64 + lane;
            const bool asc = (s & k) == 0;
            unsigned long long x = key[r], y = key[rp];
            const bool sw = asc ? (x > y) : (x < y);
            key[r] = sw ? y : x;
            key[rp] = sw ? x : y;
        }
    }
}

// Ascending sort of 64*R keys held as key[r] at position r*64 + lane.
template <int R>
__device__ __forceinline__ void wave_bitonic_sort(unsigned long long (&key)[4]) {
    const int lane = lane_id();
#pragma unroll
    for (int k = 2; k <= 64 * R; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            if (j >= 64) {
                bitonic_reg_step<R>(key, k, j, lane);
            } else {
                switch (j) {
                    case 32: bitonic_lane_step<R, 32>(key, k, lane); break;
                    case 16: bitonic_lane_step<R, 16>(key, k, lane); break;
                    case 8: bitonic_lane_step<R, 8>(key, k, lane); break;
                    case 4: bitonic_lane_step<R, 4>(key, k, lane); break;
                    case 2: bitonic_lane_step<R, 2>(key, k, lane); break;
                    default: bitonic_lane_step<R, 1>(key, k, lane); break;
                }
            }
        }
    }
}

constexpr unsigned long long kNoKey = ~0ull;

__global__ __launch_bounds__(kBlock) void k_esc(KArgs a) {
    __shared__ EscSmem smem[kBlock / 64];
    if (a.hdr->err) return;
    const int lane = lane_id();
    EscSmem &S = smem[threadIdx.x >> 6];

    // group numbering over the sort-merge sub-bins
    int bstart[kEscBins], bcnt[kEscBins], gstart[kEscBins + 1];
    {
        int run = 0;
        for (int b = 0; b < BIN_ESC0; ++b) run += a.hdr->bin_count[b];
        int gr = 0;
#pragma unroll
        for (int i = 0; i < kEscBins; ++i) {
            bstart[i] = run;
            bcnt[i] = a.hdr->bin_count[BIN_ESC0 + i];
            run += bcnt[i];
            gstart[i] = gr;
            gr += ceil_div(bcnt[i], 64 >> i);
        }
        gstart[kEscBins] = gr;
    }
    const int ngroups = gstart[kEscBins];
    const int wstride = gridDim.x * (kBlock / 64);
    for (int gi = blockIdx.x * (kBlock / 64) + (threadIdx.x >> 6); gi < ngroups; gi += wstride) {
        int sb = 0;
#pragma unroll
        for (int i = 1; i < kEscBins; ++i) sb += gi >= gstart[i];
        int G = 64, first = 0, cntb = 0, gs = 0;
#pragma unroll
        for (int i = 0; i < kEscBins; ++i)
            if (i == sb) { G = 64 >> i; first = bstart[i]; cntb = bcnt[i]; gs = gstart[i]; }
        const int lg = gi - gs;
        const int ncols = min(G, cntb - lg * G);
        first += lg * G;

        // ---- the group's columns, one per lane
        int g = 0, op = 0;
        if (lane < ncols) {
            g = a.binlist[first + lane].x;
            op = a.op[g];
            S.cbase[lane] = a.colprod[g];
        }
        const int incl = wave_incl_scan(op);
        const int E = wave_bcast(incl, 63);
        S.goff[lane] = incl - op;
        S.cnt[lane] = 0;
        if (E > kEscMaxProducts) {  // cannot happen for unchanged inputs
            if (lane == 0) atomicOr(&a.hdr->err, ERR_GROUP);
            continue;
        }
        wave_sync_lds();

        // ---- keys (column, row, e) of the group's products
        unsigned long long key[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int e = lane + 64 * r;
            key[r] = kNoKey;
            if (e < E) {
                const int cc = last_le(S.goff, ncols, e);
                const int row = a.prow[S.cbase[cc] + (e - S.goff[cc])];
                key[r] = ((unsigned long long)cc << 40) | ((unsigned long long)row << 8) |
                         (unsigned long long)e;
            }
        }
        const int R = E <= 64 ? 1 : (E <= 128 ? 2 : 4);
        if (R == 1) wave_bitonic_sort<1>(key);
        else if (R == 2) wave_bitonic_sort<2>(key);
        else wave_bitonic_sort<4>(key);
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (r < R) S.sk[r * 64 + lane] = key[r];
        wave_sync_lds();

        // ---- compress: run heads, run index of every sorted key
        bool head[4];
        int run[4];
        int before = 0;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int s = r * 64 + lane;
            head[r] = false;
            if (r < R && key[r] != kNoKey) {
                const unsigned long long prev = s > 0 ? S.sk[s - 1] : kNoKey;
                head[r] = (prev >> 8) != (key[r] >> 8);
            }
            const unsigned long long m = ballot(head[r]);
            run[r] = before + popc64(m & mask_lt()) + (head[r] ? 0 : -1);
            before += popc64(m);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            if (!head[r]) continue;
            const int s = r * 64 + lane;
            const int cc = (int)(key[r] >> 40);
            S.rh[run[r]] = s;
            const unsigned long long prev = s > 0 ? S.sk[s - 1] : kNoKey;
            if ((prev >> 40) != (unsigned long long)cc) S.cnt[cc] = run[r];
        }
        if (lane == 0) S.cnt[ncols] = before;
        wave_sync_lds();
        if (lane < ncols) a.gnnz[g] = S.cnt[lane + 1] - S.cnt[lane];
        // the largest occurrence index of the group (a device atomic only when
        // it raises the value already there)
        const int nlater = E - before;
        if (nlater > 0) {
            int kmax = 0;
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (r < R && key[r] != kNoKey) kmax = max(kmax, r * 64 + lane - S.rh[run[r]]);
#pragma unroll
            for (int dd = 32; dd >= 1; dd >>= 1)
                kmax = max(kmax, __builtin_amdgcn_ds_bpermute((lane ^ dd) << 2, kmax));
            if (lane == 0 && kmax > __atomic_load_n(&a.hdr->later_maxk, __ATOMIC_RELAXED))
                atomicMax(&a.hdr->later_maxk, kmax);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            if (r >= R || key[r] == kNoKey) continue;
            const int s = r * 64 + lane;
            const int cc = (int)(key[r] >> 40);
            const int e = (int)(key[r] & 255u);
            const int rank = run[r] - S.cnt[cc];
            const int k = s - S.rh[run[r]];
            const long long pe = S.cbase[cc] + (e - S.goff[cc]);
            if (k == 0) {
                a.dst[pe] = (uint32_t)rank;
            } else {
                // index among the column's later products: later keys before
                // this one in sorted order, minus those of the earlier columns
                // of the group (their products minus their entries)
                a.dst[pe] = kDstLater | (uint32_t)rank;
                a.lk[pe] = k;
                a.lr[pe] = (s - run[r] - 1) - (S.goff[cc] - S.cnt[cc]);
            }
        }
    }
}

hipError_t launch_esc(const KArgs &a, int grid, hipStream_t s) {
    if (grid <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_esc, dim3(grid), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

}  // namespace spg
