// Wavefront sort-merge accumulator for the lightest columns: expand, sort,
// compress (ESC, Section 4), one 64-lane wavefront per group of columns.
//
// A group holds up to 64 columns whose products and stored B entries each add
// up to at most 256. The wavefront
//   1. expands every product of the group in the order the sequential SPA of
//      Algorithm 1 meets them (B entries in storage order, then the rows of
//      the A column in storage order); e is the position in that order;
//   2. sorts the keys (column, row, e) with a register bitonic network whose
//      lane exchanges use DPP, ds_swizzle and ds_bpermute;
//   3. compresses: the first key of every (column, row) run sums the run's
//      products in e order, which is the order Algorithm 1 adds them, so the
//      values are bit-identical to it; its rank inside the column is its
//      output position (rows come out ascending).
// The symbolic mode runs steps 1-3 without values and counts the runs.
#include "devutil.h"

namespace spg {

template <typename V, bool NUM>
struct EscSmem {
    int boff[65];   // first B-entry index of each column in the group
    int cbs[64];    // first stored B entry of each column
    int cpid[64];   // problem of each column
    int cbase[64];  // output position of each column (numeric)
    int clen[64];   // nnz of each output column (numeric)
    int cnt[64];    // symbolic: runs per column; numeric: first run index
    union {
        struct {
            int tacp[kEscMaxProducts];       // A column start per B entry
            int teoff[kEscMaxProducts + 1];  // first product index per B entry
            unsigned char tc[kEscMaxProducts];
            V tb[NUM ? kEscMaxProducts : 1];  // B value per entry
        } ex;
        unsigned long long sk[kEscMaxProducts];  // sorted keys
    } u;
    V pv[NUM ? kEscMaxProducts : 1];  // product value by expansion position
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

template <typename V, bool NUM>
__global__ __launch_bounds__(kBlock) void k_esc(KArgs a) {
    __shared__ EscSmem<V, NUM> smem[kBlock / 64];
    if (a.hdr->err) return;
    const int lane = lane_id();
    EscSmem<V, NUM> &S = smem[threadIdx.x >> 6];

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

        // ---- level 1: the group's columns, one per lane
        int g = 0, nb = 0;
        if (lane < ncols) {
            const int4 ent = a.binlist[first + lane];
            g = ent.x;
            nb = ent.z;
            const int pid = find_prob(a, g);
            const Prob d = get_prob(a, pid);
            const int j = g - d.col0;
            S.cbs[lane] = ent.y;
            S.cpid[lane] = pid;
            if (NUM) {
                const int c0 = d.ccp[j];
                S.cbase[lane] = c0;
                S.clen[lane] = d.ccp[j + 1] - c0;
            }
        }
        const int incl = wave_incl_scan(nb);
        const int TB = wave_bcast(incl, 63);
        S.boff[lane] = incl - nb;
        S.cnt[lane] = 0;
        if (TB > kEscMaxProducts) {  // cannot happen for unchanged inputs
            if (lane == 0) atomicOr(&a.hdr->err, ERR_GROUP);
            continue;
        }
        wave_sync_lds();

        // ---- level 2: stored B entries of the group, in storage order
        int zr[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int t = lane + 64 * r;
            zr[r] = 0;
            if (t < TB) {
                const int cc = last_le(S.boff, ncols, t);
                const int p = S.cbs[cc] + t - S.boff[cc];
                const Prob d = get_prob(a, S.cpid[cc]);
                const int2 ez = a.E[d.ebase + p];  // (A column start, length), checked
                S.u.ex.tc[t] = (unsigned char)cc;
                S.u.ex.tacp[t] = ez.x;
                zr[r] = ez.y;
                if (NUM) S.u.ex.tb[t] = ((const V *)d.bv)[p];
            }
        }
        int E = 0;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int t = lane + 64 * r;
            const int inc = wave_incl_scan(zr[r]);
            if (t < TB) S.u.ex.teoff[t] = E + inc - zr[r];
            E += wave_bcast(inc, 63);
        }
        if (E > kEscMaxProducts) {
            if (lane == 0) atomicOr(&a.hdr->err, ERR_GROUP);
            continue;
        }
        wave_sync_lds();

        // ---- level 3: products, key = (column, row, e)
        unsigned long long key[4];
        int bad = 0;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int e = lane + 64 * r;
            key[r] = kNoKey;
            if (e < E) {
                const int tt = last_le(S.u.ex.teoff, TB, e);
                const int q = S.u.ex.tacp[tt] + e - S.u.ex.teoff[tt];
                const int cc = S.u.ex.tc[tt];
                const Prob d = get_prob(a, S.cpid[cc]);
                const int row = d.ari[q];
                if (row < 0 || row >= d.m) {
                    bad = 1;
                } else {
                    key[r] = ((unsigned long long)cc << 40) | ((unsigned long long)row << 8) |
                             (unsigned long long)e;
                    if (NUM) S.pv[e] = ((const V *)d.av)[q] * S.u.ex.tb[tt];
                }
            }
        }
        if (ballot(bad)) {
            if (lane == 0) atomicOr(&a.hdr->err, ERR_CSC);
            continue;
        }
        const int R = E <= 64 ? 1 : (E <= 128 ? 2 : 4);
        if (R == 1) wave_bitonic_sort<1>(key);
        else if (R == 2) wave_bitonic_sort<2>(key);
        else wave_bitonic_sort<4>(key);
        wave_sync_lds();
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (r < R) S.u.sk[r * 64 + lane] = key[r];
        wave_sync_lds();

        // ---- compress
        bool head[4];
        int hidx[4];
        int before = 0;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int s = r * 64 + lane;
            head[r] = false;
            if (r < R && key[r] != kNoKey) {
                const unsigned long long prev = s > 0 ? S.u.sk[s - 1] : kNoKey;
                head[r] = (prev >> 8) != (key[r] >> 8);
            }
            const unsigned long long m = ballot(head[r]);
            hidx[r] = before + popc64(m & mask_lt());
            before += popc64(m);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            if (!head[r]) continue;
            const int s = r * 64 + lane;
            const int cc = (int)(key[r] >> 40);
            if (NUM) {
                const unsigned long long prev = s > 0 ? S.u.sk[s - 1] : kNoKey;
                if ((prev >> 40) != (unsigned long long)cc) S.cnt[cc] = hidx[r];
            } else {
                atomicAdd(&S.cnt[cc], 1);
            }
        }
        wave_sync_lds();
        if (!NUM) {
            if (lane < ncols) a.gnnz[g] = S.cnt[lane];
            continue;
        }
        int oob = 0;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            if (!head[r]) continue;
            const int s = r * 64 + lane;
            const unsigned long long kr = key[r] >> 8;
            const int cc = (int)(key[r] >> 40);
            V acc = V(0);
            for (int t = s; t < E; ++t) {
                const unsigned long long k2 = S.u.sk[t];
                if ((k2 >> 8) != kr) break;
                acc = acc + S.pv[(int)(k2 & 255u)];
            }
            const int rank = hidx[r] - S.cnt[cc];
            if (rank >= S.clen[cc]) { oob = 1; continue; }
            const int out = S.cbase[cc] + rank;
            const Prob d = get_prob(a, S.cpid[cc]);
            d.cri[out] = (int)((key[r] >> 8) & 0x7fffffffull);
            ((V *)d.cv)[out] = acc;
        }
        if (ballot(oob) && lane == 0) atomicOr(&a.hdr->err, ERR_GROUP);
    }
}

hipError_t launch_esc(const KArgs &a, bool numeric, bool f64, int grid, hipStream_t s) {
    if (grid <= 0) return hipSuccess;
    if (f64) {
        if (numeric) hipLaunchKernelGGL((k_esc<double, true>), dim3(grid), dim3(kBlock), 0, s, a);
        else hipLaunchKernelGGL((k_esc<double, false>), dim3(grid), dim3(kBlock), 0, s, a);
    } else {
        if (numeric) hipLaunchKernelGGL((k_esc<float, true>), dim3(grid), dim3(kBlock), 0, s, a);
        else hipLaunchKernelGGL((k_esc<float, false>), dim3(grid), dim3(kBlock), 0, s, a);
    }
    return hipGetLastError();
}

}  // namespace spg
