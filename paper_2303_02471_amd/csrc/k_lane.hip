// Lane-per-column hash accumulator: the paper's HASH (Section 3.2) mapped one
// output column per lane, as its vector algorithms map one column per vector
// element. Optional (SPGEMM_LANE_HASH): it takes the wavefront sort-merge
// sub-bins of at most 64 products, so the two can be compared on the same
// columns.
//
// Every lane owns a private open-addressing table of H = 2 S slots in LDS
// (S: the sub-bin's largest product count, so the load factor stays at or
// below 1/2), keyed by row with linear probing from a multiplicative hash.
// Inserting the column's products in Algorithm 1's order gives each product
// its slot and its occurrence index k (the count of earlier products of the
// same row). The paper stores each table sorted; here the lane ranks its
// distinct rows by counting smaller keys, which gives every row its output
// rank and the number of later products of smaller rows, so the outputs are
// exactly those of the other accumulators: the rank as destination (marked
// for k > 0), k, and the index among the column's later products in
// sorted-key order.
#include "devutil.h"

namespace spg {

constexpr int kLaneWave = 64;  // one wavefront per workgroup: lanes share nothing

template <int LS>
struct LaneSmem {
    static constexpr int S = 1 << LS, H = 2 * S;
    int key[H * kLaneWave];             // slot h of lane l at h * 64 + l
    uint8_t cnt[H * kLaneWave];         // products of the slot's row so far
    uint8_t rank[H * kLaneWave];        // rank of the slot's row among the column's rows
    uint8_t lbefore[H * kLaneWave];     // later products of smaller rows
    uint8_t used[S * kLaneWave];        // the used slots, in order of first use
    uint16_t ps[S * kLaneWave];         // per product: slot | k << 8
};

template <int LS>
__global__ __launch_bounds__(kLaneWave) void k_lane(KArgs a) {
    using Sm = LaneSmem<LS>;
    constexpr int S = Sm::S, H = Sm::H;
    __shared__ Sm L;
    if (__atomic_load_n(&a.hdr->err, __ATOMIC_RELAXED) != 0) return;
    const int lane = threadIdx.x;
    const int sub = LS - 2;
    int start = 0;
    for (int b = 0; b < BIN_ESC0 + sub; ++b) start += a.hdr->bin_count[b];
    const int ncols = a.hdr->bin_count[BIN_ESC0 + sub];
    int kmax = 0;
    // the grid may be planned from an earlier call's column count: every
    // lane strides over the device count
    for (int ci = blockIdx.x * kLaneWave + lane; ci < ncols; ci += gridDim.x * kLaneWave) {
        const int g = a.binlist[start + ci].x;
        const int op = a.op[g];
        const long long pbase = a.colprod[g];
        if (op > S) {  // more than planned: cannot happen for unchanged inputs
            atomicOr(&a.hdr->err, ERR_GROUP);
        } else {
            auto K = [&](int h) -> int & { return L.key[h * kLaneWave + lane]; };
            auto C = [&](int h) -> uint8_t & { return L.cnt[h * kLaneWave + lane]; };
            for (int h = 0; h < H; ++h) {
                K(h) = -1;
                C(h) = 0;
            }
            int d = 0;
            for (int e = 0; e < op; ++e) {
                const int r = a.prow[pbase + e];
                int h = (int)(((unsigned)r * 2654435761u) >> (32 - (LS + 1)));
                while (K(h) != -1 && K(h) != r) h = (h + 1) & (H - 1);
                if (K(h) == -1) {
                    K(h) = r;
                    L.used[d * kLaneWave + lane] = (uint8_t)h;
                    ++d;
                }
                const int k = C(h);
                C(h) = (uint8_t)(k + 1);
                L.ps[e * kLaneWave + lane] = (uint16_t)(h | (k << 8));
            }
            // rank of each distinct row, and the later products of smaller rows
            for (int i = 0; i < d; ++i) {
                const int h = L.used[i * kLaneWave + lane];
                const int r = K(h);
                int rk = 0, lb = 0;
                for (int j = 0; j < d; ++j) {
                    const int h2 = L.used[j * kLaneWave + lane];
                    if (K(h2) < r) {
                        ++rk;
                        lb += C(h2) - 1;
                    }
                }
                L.rank[h * kLaneWave + lane] = (uint8_t)rk;
                L.lbefore[h * kLaneWave + lane] = (uint8_t)lb;
            }
            for (int e = 0; e < op; ++e) {
                const int v = L.ps[e * kLaneWave + lane];
                const int h = v & 255, k = v >> 8;
                const int rk = L.rank[h * kLaneWave + lane];
                if (k == 0) {
                    a.dst[pbase + e] = (uint32_t)rk;
                } else {
                    a.dst[pbase + e] = kDstLater | (uint32_t)rk;
                    a.lk[pbase + e] = k;
                    a.lr[pbase + e] = L.lbefore[h * kLaneWave + lane] + k - 1;
                    kmax = max(kmax, k);
                }
            }
            a.gnnz[g] = d;
        }
    }
    // every lane reaches this reduction (no early exit above)
#pragma unroll
    for (int dd = 32; dd >= 1; dd >>= 1)
        kmax = max(kmax, __builtin_amdgcn_ds_bpermute((lane ^ dd) << 2, kmax));
    if (lane == 0 && kmax > __atomic_load_n(&a.hdr->later_maxk, __ATOMIC_RELAXED))
        atomicMax(&a.hdr->later_maxk, kmax);
}

hipError_t launch_lane(const KArgs &a, int sub, int ncols, hipStream_t s) {
    if (ncols <= 0) return hipSuccess;
    const dim3 grid(ceil_div(ncols, kLaneWave));
    switch (sub) {
        case 0: hipLaunchKernelGGL((k_lane<2>), grid, dim3(kLaneWave), 0, s, a); break;
        case 1: hipLaunchKernelGGL((k_lane<3>), grid, dim3(kLaneWave), 0, s, a); break;
        case 2: hipLaunchKernelGGL((k_lane<4>), grid, dim3(kLaneWave), 0, s, a); break;
        case 3: hipLaunchKernelGGL((k_lane<5>), grid, dim3(kLaneWave), 0, s, a); break;
        case 4: hipLaunchKernelGGL((k_lane<6>), grid, dim3(kLaneWave), 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace spg
