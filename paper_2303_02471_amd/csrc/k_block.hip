// Workgroup accumulator of the columns with more products than the wavefront
// sort-merge takes: one workgroup per column, an LDS table per row window.
//
// The column's rows [lo, hi] (from its products) are cut into W windows of
// equal row span, W chosen so that every window plans at most `cap` distinct
// rows. A window whose span fits the table is accumulated by direct indexing
// -- slot = row - x, the SPA of Section 2.2 restricted to the window. Other
// windows use the hash accumulator of Section 3.2 with a table of about twice
// the planned distinct rows (its size adaptation), an order-preserving hash
// home(r) = floor((r - x) * H / span) and linear probing that never wraps. The
// table then comes out sorted run by run: every run of occupied slots only
// holds rows whose home slots lie in it, and every row of a run lies between
// the rows of the runs before and after it. The rank of a row is therefore
// the number of occupied slots before its run plus the number of smaller rows
// inside its run. A window whose distinct rows overrun the table's overflow
// area is split in halves and each half redone (linear probing's occupied set
// does not depend on insertion order, so the split is deterministic).
//
// A slot holds (row << 32 | e) with e the position of the product in the
// order Algorithm 1 meets it (stored B entries in storage order, then the
// rows of the selected A column in storage order): the first insert of a row
// claims the slot with a compare-and-swap, later ones keep the smallest e
// with an atomic minimum. So, per window:
//   1. clear; insert every product whose row is in the window;
//   2. a product is the first of its output entry when its e is the slot's;
//   3. ranks: occupancy prefix over the slots plus in-run order, stored in the
//      slot's low word;
//   4. destinations: every product gets the rank of its entry in the column
//      (earlier windows' entries before it); a product that is not the first
//      of its entry is marked and gets its occurrence index k (its position
//      among the entry's products in Algorithm 1's order) and an index among
//      the column's later products, resolved chunk by chunk in product order:
//      products of one chunk that share an entry offer (round, position) to
//      the entry with an LDS atomic maximum, the earliest wins its k and
//      retires, the rest retry.
// Columns of at most T * PER products keep their rows in registers; larger
// ones stream them again for every pass (and plan half the table, the other
// half holding the occurrence counters).
#include "devutil.h"

namespace spg {

template <int CLS>
struct BlkCfg;
// T threads, TC 8-byte LDS slots, PER products per thread held in registers
template <>
struct BlkCfg<0> { static constexpr int T = 256, TC = 2048, PER = 2; };
template <>
struct BlkCfg<1> { static constexpr int T = 256, TC = 4096, PER = 4; };
template <>
struct BlkCfg<2> { static constexpr int T = 512, TC = 8192, PER = 4; };
template <>
struct BlkCfg<3> { static constexpr int T = 1024, TC = 12288, PER = 4; };
template <>
struct BlkCfg<4> { static constexpr int T = 1024, TC = 18432, PER = 8; };

constexpr unsigned long long kEmpty = ~0ull;
constexpr unsigned kEmptyHi = ~0u;
constexpr int kSplitDepth = 48;

template <int CLS>
struct BlkSmem {
    static constexpr int T = BlkCfg<CLS>::T, TC = BlkCfg<CLS>::TC;
    unsigned long long tab[TC];
    int scan_tmp[T / 64 + 1];
    int stk_lo[kSplitDepth], stk_hi[kSplitDepth];
    int s_min, s_max, s_nlater, s_lcur, s_kmax;
};

// overflow slots behind a hash table of h home slots, within the capacity
__device__ __forceinline__ int blk_pad(int h, int cap) { return min(min(256, h / 4 + 16), cap - h); }

template <int CLS>
__global__ __launch_bounds__(BlkCfg<CLS>::T) void k_block(KArgs a) {
    constexpr int T = BlkCfg<CLS>::T, TC = BlkCfg<CLS>::TC, PER = BlkCfg<CLS>::PER;
    constexpr int CH = T * PER;
    constexpr int PB = T <= 256 ? 8 : (T <= 512 ? 9 : 10);  // bits of a position in a chunk
    static_assert((1 << PB) >= T, "chunk positions fit the stamp");
    constexpr unsigned kRoundLimit = (1u << (32 - PB)) - 2;
    __shared__ BlkSmem<CLS> S;
    if (__syncthreads_or(__atomic_load_n(&a.hdr->err, __ATOMIC_RELAXED) != 0))
        return;  // every thread takes the same branch
    const int tid = threadIdx.x;
    unsigned *hw = (unsigned *)S.tab;  // hw[2s]: low word (e, then rank); hw[2s + 1]: row
    int first = 0;
    for (int b = 0; b < BIN_BLK0 + CLS; ++b) first += a.hdr->bin_count[b];
    const int n = a.hdr->bin_count[BIN_BLK0 + CLS];
    int err = 0, kmax = 0;
    bool abort = false;  // workgroup-uniform: a window could not be split further
    if (tid == 0) S.s_kmax = 0;

    for (int li = blockIdx.x; li < n; li += gridDim.x) {
        const int g = a.binlist[first + li].x;
        const int op = a.op[g];
        const long long pbase = a.colprod[g];
        const int *__restrict__ prow = a.prow + pbase;
        uint32_t *__restrict__ dstp = a.dst + pbase;
        const bool fits = op <= CH;
        const int tcap = fits ? TC : TC / 2;  // table slots
        int *cnt = fits ? (int *)S.tab : (int *)(S.tab + TC / 2);
        unsigned *stamps = (unsigned *)(cnt + tcap);

        // ---- rows (registers when they fit) and the column's row range
        int rr[PER];
        if (fits) {
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                const int e = u * T + tid;
                rr[u] = e < op ? prow[e] : -1;
            }
        }
        if (tid == 0) {
            S.s_min = 0x7fffffff;
            S.s_max = -1;
        }
        __syncthreads();
        {
            int mn = 0x7fffffff, mx = -1;
            if (fits) {
#pragma unroll
                for (int u = 0; u < PER; ++u)
                    if (rr[u] >= 0) { mn = min(mn, rr[u]); mx = max(mx, rr[u]); }
            } else {
                for (int e = tid; e < op; e += T) {
                    const int r = prow[e];
                    mn = min(mn, r);
                    mx = max(mx, r);
                }
            }
#pragma unroll
            for (int d = 32; d >= 1; d >>= 1) {
                mn = min(mn, __builtin_amdgcn_ds_bpermute((lane_id() ^ d) << 2, mn));
                mx = max(mx, __builtin_amdgcn_ds_bpermute((lane_id() ^ d) << 2, mx));
            }
            if (lane_id() == 0) {
                atomicMin(&S.s_min, mn);
                atomicMax(&S.s_max, mx);
            }
        }
        __syncthreads();
        const int lo = S.s_min, span = S.s_max + 1 - S.s_min;  // op > 0: at least one row

        // ---- row windows
        const int hmax = tcap - min(256, tcap / 8);  // largest table (home slots)
        int cap = hmax / 2;
        if (a.tune.hash_cap > 0) cap = min(cap, a.tune.hash_cap);
        int W = op <= cap ? 1 : ceil_div(op, cap);
        if (W > span) W = span;
        const int plan = max(64, min(hmax, 2 * ceil_div(op, W)));
        const int dlim = min(tcap, a.tune.dense_rows > 0 ? a.tune.dense_rows : tcap);
        int total = 0;   // entries of the earlier windows
        int ltotal = 0;  // later products of the earlier windows
        int wflags = 0;  // WinFlags of the column

        for (int w = 0; w < W; ++w) {
            if (tid == 0) {
                S.stk_lo[0] = lo + (int)((long long)w * span / W);
                S.stk_hi[0] = lo + (int)((long long)(w + 1) * span / W);
            }
            int sp = 1;
            __syncthreads();
            while (sp > 0) {
                --sp;
                const int x = S.stk_lo[sp], y = S.stk_hi[sp];
                const int sw = y - x;
                const bool direct = op >= a.tune.t_dense && sw <= dlim && sw <= 4 * plan;
                const int nslot = direct ? sw : plan;
                const int nst = nslot + (direct ? 0 : blk_pad(nslot, tcap));
                const unsigned long long scale =
                    direct ? 0ull : (((unsigned long long)nslot << 32) / (unsigned long long)sw);
                auto home = [&](int r) -> int {
                    return direct ? r - x
                                  : (int)(((unsigned long long)(unsigned)(r - x) * scale) >> 32);
                };
                // slot of a row already in the table
                auto lookup = [&](int r) -> int {
                    int s = home(r);
                    while (s < nst && hw[2 * s + 1] != (unsigned)r) ++s;
                    return s;
                };
                // ---- 1. clear, insert
                for (int s = tid; s < nst; s += T) S.tab[s] = kEmpty;
                if (tid == 0) {
                    S.s_nlater = 0;
                    S.s_lcur = 0;
                }
                __syncthreads();
                auto insert = [&](int r, int e) -> int {  // slot, or -1 when the table overruns
                    int s = home(r);
                    const unsigned long long key =
                        ((unsigned long long)(unsigned)r << 32) | (unsigned)e;
                    while (s < nst) {
                        unsigned long long cur = S.tab[s];
                        if ((unsigned)(cur >> 32) == kEmptyHi) {
                            cur = atomicCAS(&S.tab[s], kEmpty, key);
                            if (cur == kEmpty) return s;
                        }
                        if ((unsigned)(cur >> 32) == (unsigned)r) {
                            atomicMin(&S.tab[s], key);
                            return s;
                        }
                        ++s;
                    }
                    return -1;
                };
                int slot[PER];     // slot of each product (-1: not in the window), then its rank
                unsigned fst = 0;  // bit u: product u is the first of its entry
                static_assert(PER <= 32, "first-product bits");
                int fail = 0;
                if (fits) {
#pragma unroll
                    for (int u = 0; u < PER; ++u) {
                        slot[u] = -1;
                        const int r = rr[u];
                        if (r >= x && r < y) {
                            const int s = insert(r, u * T + tid);
                            if (s < 0) fail = 1;
                            slot[u] = s;
                        }
                    }
                } else {
                    for (int e0 = 0; e0 < op; e0 += CH) {
                        int r[PER];
#pragma unroll
                        for (int u = 0; u < PER; ++u) {
                            const int e = e0 + u * T + tid;
                            r[u] = e < op ? prow[e] : -1;
                        }
#pragma unroll
                        for (int u = 0; u < PER; ++u)
                            if (r[u] >= x && r[u] < y && insert(r[u], e0 + u * T + tid) < 0) fail = 1;
                    }
                }
                if (__syncthreads_or(fail)) {
                    // split the window; the left half is taken first
                    if (sw <= 1 || sp + 2 > kSplitDepth) {  // cannot happen: one row always fits
                        abort = true;
                        break;
                    }
                    const int mid = x + sw / 2;
                    if (tid == 0) {
                        S.stk_lo[sp] = mid; S.stk_hi[sp] = y;
                        S.stk_lo[sp + 1] = x; S.stk_hi[sp + 1] = mid;
                    }
                    wflags |= WF_SPLIT;
                    sp += 2;
                    __syncthreads();
                    continue;
                }
                wflags |= direct ? WF_DIRECT : WF_HASH;

                // ---- 2. first product of every entry; later products counted
                int nl = 0;
                if (fits) {
#pragma unroll
                    for (int u = 0; u < PER; ++u) {
                        if (slot[u] < 0) continue;
                        const bool f = hw[2 * slot[u]] == (unsigned)(u * T + tid);
                        fst |= (unsigned)f << u;
                        nl += !f;
                    }
                } else {
                    // the mark (0 first, 1 later) waits in the destination entry
                    for (int e = tid; e < op; e += T) {
                        const int r = prow[e];
                        if (r < x || r >= y) continue;
                        const int s = lookup(r);
                        const bool f = s < nst && hw[2 * s] == (unsigned)e;
                        dstp[e] = f ? 0u : 1u;
                        nl += !f;
                    }
                }
                nl = wave_sum(nl);
                if (lane_id() == 0 && nl) atomicAdd(&S.s_nlater, nl);
                __syncthreads();

                // ---- 3. ranks into the slots' low words
                int distinct;
                {
                    // consecutive slots per thread; an odd count keeps the
                    // threads of a wavefront on distinct LDS banks
                    const int per = ceil_div(nst, T) | 1;
                    const int s0 = min(nst, tid * per), s1 = min(nst, s0 + per);
                    int mycnt = 0;
                    for (int sl = s0; sl < s1; ++sl) mycnt += hw[2 * sl + 1] != kEmptyHi;
                    int run = wg_excl_scan<T>(mycnt, S.scan_tmp, distinct);
                    int cs = -1, ce = -1;  // bounds of the current run of occupied slots
                    for (int sl = s0; sl < s1; ++sl) {
                        const unsigned r = hw[2 * sl + 1];
                        if (r == kEmptyHi) { cs = -1; continue; }
                        int rank = run;
                        if (!direct) {
                            if (cs < 0) {
                                cs = sl;
                                while (cs > 0 && hw[2 * (cs - 1) + 1] != kEmptyHi) --cs;
                                ce = sl + 1;
                                while (ce < nst && hw[2 * ce + 1] != kEmptyHi) ++ce;
                            }
                            int less = 0;
                            for (int t = cs; t < ce; ++t) less += hw[2 * t + 1] < r;
                            rank = run - (sl - cs) + less;
                        }
                        hw[2 * sl] = (unsigned)rank;
                        ++run;
                    }
                }
                __syncthreads();

                // ---- 4. destinations
                const int nlater = S.s_nlater;
                if (fits) {
#pragma unroll
                    for (int u = 0; u < PER; ++u) {
                        if (slot[u] < 0) continue;
                        slot[u] = total + (int)hw[2 * slot[u]];  // now the rank
                        if ((fst >> u) & 1u) dstp[u * T + tid] = (uint32_t)slot[u];
                    }
                }
                if (fits && nlater) __syncthreads();  // the table is read: its memory is reused
                if (nlater) {
                    for (int i = tid; i < distinct; i += T) {
                        cnt[i] = 0;
                        stamps[i] = 0u;
                    }
                    __syncthreads();
                }
                unsigned round = 0;
                // occurrence indices of the pending later products of one chunk of T
                auto settle = [&](bool pend, int idx, int rank, int e) {
                    if (pend && (idx < 0 || idx >= distinct)) {  // cannot happen
                        err = ERR_GROUP;
                        pend = false;
                    }
                    if (!__syncthreads_or(pend)) return;
                    if (round + T + 1 > kRoundLimit) {  // keep rounds inside their stamp bits
                        for (int i = tid; i < distinct; i += T) stamps[i] = 0u;
                        round = 0;
                        __syncthreads();
                    }
                    const unsigned pos = (unsigned)(T - 1 - tid);
                    bool more;
                    do {
                        ++round;
                        const unsigned mine = (round << PB) | pos;
                        if (pend) atomicMax(&stamps[idx], mine);
                        __syncthreads();
                        if (pend && stamps[idx] == mine) {
                            const int k = ++cnt[idx];
                            const int lix = atomicAdd(&S.s_lcur, 1);
                            if (lix < nlater) {
                                dstp[e] = kDstLater | (uint32_t)rank;
                                a.lk[pbase + e] = k;
                                a.lr[pbase + e] = ltotal + lix;
                                kmax = max(kmax, k);
                            } else {
                                err = ERR_GROUP;
                            }
                            pend = false;
                        }
                        more = __syncthreads_or(pend);
                    } while (more);
                };
                if (nlater) {
                    if (fits) {
#pragma unroll
                        for (int u = 0; u < PER; ++u)
                            settle(slot[u] >= 0 && !((fst >> u) & 1u), slot[u] - total, slot[u],
                                   u * T + tid);
                    } else {
                        for (int e0 = 0; e0 < op; e0 += T) {
                            const int e = e0 + tid;
                            bool pend = false;
                            int rank = 0;
                            if (e < op) {
                                const int r = prow[e];
                                if (r >= x && r < y) {
                                    const int s = lookup(r);
                                    rank = total + (s < nst ? (int)hw[2 * s] : 0);
                                    if (dstp[e] == 0u) dstp[e] = (uint32_t)rank;
                                    else pend = true;
                                }
                            }
                            settle(pend, rank - total, rank, e);
                        }
                    }
                } else if (!fits) {
                    for (int e = tid; e < op; e += T) {
                        const int r = prow[e];
                        if (r < x || r >= y) continue;
                        const int s = lookup(r);
                        dstp[e] = (uint32_t)(total + (s < nst ? (int)hw[2 * s] : 0));
                    }
                }
                total += distinct;
                ltotal += nlater;
                __syncthreads();
            }
            if (abort) break;
        }
        if (tid == 0) {
            a.gnnz[g] = total;
            a.binw[g] = (BIN_BLK0 + CLS) | (wflags << 8);
        }
        __syncthreads();
        if (abort) break;
    }
    if (abort) err = ERR_GROUP;
    if (err) atomicOr(&a.hdr->err, err);
    // the largest k: one device atomic per workgroup at most, and only when it
    // raises the value already there
    if (kmax) atomicMax(&S.s_kmax, kmax);
    __syncthreads();
    if (tid == 0 && S.s_kmax > __atomic_load_n(&a.hdr->later_maxk, __ATOMIC_RELAXED))
        atomicMax(&a.hdr->later_maxk, S.s_kmax);
}

hipError_t launch_block(const KArgs &a, int cls, int grid, hipStream_t s) {
    if (grid <= 0) return hipSuccess;
#define SPG_LAUNCH(C) hipLaunchKernelGGL((k_block<C>), dim3(grid), dim3(BlkCfg<C>::T), 0, s, a)
    switch (cls) {
        case 0: SPG_LAUNCH(0); break;
        case 1: SPG_LAUNCH(1); break;
        case 2: SPG_LAUNCH(2); break;
        case 3: SPG_LAUNCH(3); break;
        default: SPG_LAUNCH(4); break;
    }
#undef SPG_LAUNCH
    return hipGetLastError();
}

}  // namespace spg
