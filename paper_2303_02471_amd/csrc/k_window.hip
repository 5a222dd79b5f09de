// Symbolic accumulators of the heavier columns, one workgroup per (column,
// row window):
//
//   DENSE: the SPA of Section 2.2 restricted to LDS -- one slot per row of the
//          window plus an occupancy bitmap; the rank of a row is the number
//          of occupied rows below it.
//   HASH:  the hash accumulator of Section 3.2 -- an open-addressing table with
//          linear probing, sized per column from its product count (its
//          size adaptation). The hash is order-preserving,
//          h(i) = floor((i - lo) * H / (hi - lo)), and probes never wrap, so
//          every run of occupied slots only holds rows whose home slots lie in
//          it, and all of them lie between the rows of the runs before and
//          after it: the rank of a row is the number of occupied slots before
//          its run plus the number of smaller rows inside its run.
//          Three instantiations differ only in the largest table (LDS
//          footprint) and in the workgroup size.
//
// Pass 1 expands the window's products in the order Algorithm 1 meets them
// (stored B entries in storage order, then the rows of the selected A column
// in storage order) and inserts their rows, counting products per slot. When
// the window is the whole column it also writes each product's slot to the
// product's destination entry. After the ranks are known, pass 2 streams
// those slots (or expands the products again for a windowed or split column)
// and records the destination of every product: the rank of its row in the
// window, and for an output reached by several products the occurrence index
// k of the product among them (list order). Products of one chunk that land on the
// same slot take their k in list order: every pending product offers
// (round, position in chunk) to the slot with an LDS atomic max, the earliest
// one wins and retires; the others retry next round.
//
// A window whose distinct rows overflow the table (linear probing never
// wraps; a probe running past the table's overrun area fails) is split in
// halves and each half is redone; ranks continue across the halves.
#include "devutil.h"

namespace spg {

template <int MODE>
struct WinCfg {
    static constexpr bool DENSE = MODE == WIN_DENSE;
    static constexpr int HMAX =
        MODE == WIN_HASH_S ? kHashMaxS : (MODE == WIN_HASH_L ? kHashMaxL : kHashMax);
    static constexpr int TBL = DENSE ? kDenseRows : HMAX + hash_pad(HMAX);
    // threads per workgroup: the extra-large class fills a CU with one
    // workgroup, the large class with two
    static constexpr int T = MODE == WIN_HASH_XL ? 1024 : (MODE == WIN_HASH_L ? 512 : 256);
    static constexpr int PER = 2;  // products per thread per chunk
};

template <int MODE>
struct WinSmem {
    using C = WinCfg<MODE>;
    int keys[C::DENSE ? 1 : C::TBL];  // row held by each slot, -1 when empty
    unsigned bitmap[C::DENSE ? kDenseRows / 32 : 1];
    int wpre[C::DENSE ? kDenseRows / 32 : 1];  // occupied rows before each bitmap word
    int cnt[C::TBL];    // pass 1: products per slot; pass 2: occurrences handed out
    int rank[C::TBL];   // rank of the slot's row; bit 31 when several products reach it
    unsigned stamps[C::TBL];
    int scan_tmp[C::T / 64 + 1];
    int stk_lo[40], stk_hi[40];
    int s_count, s_prod, s_err, s_lcur, s_kmax;
    long long s_lbase;  // first place of the window's later products in the later list
};

// exclusive prefix over the workgroup (T threads); contains barriers
template <int T>
__device__ __forceinline__ int wg_excl_scan(int v, int *tmp, int &total) {
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    int inc = wave_incl_scan(v);
    if (l == 63) tmp[w] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        int run = 0;
        for (int i = 0; i < T / 64; ++i) {
            int x = tmp[i];
            tmp[i] = run;
            run += x;
        }
        tmp[T / 64] = run;
    }
    __syncthreads();
    int ex = tmp[w] + inc - v;
    total = tmp[T / 64];
    __syncthreads();
    return ex;
}

constexpr int kMulti = (int)0x80000000u;

template <int MODE>
__global__ __launch_bounds__(WinCfg<MODE>::T) void k_window(KArgs a) {
    using CF = WinCfg<MODE>;
    using SM = WinSmem<MODE>;
    constexpr bool DENSE = CF::DENSE;
    constexpr int T = CF::T, PER = CF::PER, CH = T * PER;
    // a stamp is (round << PB) | (CH - 1 - position in chunk)
    constexpr int PB = CH <= 512 ? 9 : (CH <= 1024 ? 10 : 11);
    static_assert(CH <= (1 << PB), "chunk positions must fit the stamp");
    constexpr unsigned kRoundLimit = 1u << (31 - PB);
    __shared__ SM S;
    if (a.hdr->err) return;
    const int tid = threadIdx.x;

    int istart = 0, nitems = 0, dstart = 0;
    if (DENSE) {
        for (int b = 0; b < BIN_DENSE; ++b) dstart += a.hdr->bin_count[b];
        nitems = a.hdr->bin_count[BIN_DENSE];
    } else {
        int tot = 0;
        for (int h = 0; h < kHashBins; ++h) {
            if (h == MODE - WIN_HASH_S) {
                istart = tot;
                nitems = a.hdr->item_count[h];
            }
            tot += a.hdr->item_count[h];
        }
        if (tot > a.item_cap) return;
    }

    unsigned round = 0;
    for (int s = tid; s < CF::TBL; s += T) S.stamps[s] = 0;
    __syncthreads();

    for (int li = blockIdx.x; li < nitems; li += gridDim.x) {
        const int it = istart + li;
        int g, w = 0, W = 1;
        if (DENSE) {
            g = a.binlist[dstart + li].x;
        } else {
            g = a.items[it].x;
            w = it - a.colitem[g];
            W = a.binw[g] >> 8;
        }
        const int pid = find_prob(a, g);
        const Prob d = get_prob(a, pid);
        const int op = a.op[g];
        const long long pbase = a.colprod[g];
        const int lo0 = window_lo(w, W, d.m);
        const int hi0 = window_lo(w + 1, W, d.m);
        const int H = DENSE ? 0 : hash_table_size(op, W);
        const int *__restrict__ prow = a.prow + pbase;

        int total = 0;
        if (tid == 0) {
            S.stk_lo[0] = lo0;
            S.stk_hi[0] = hi0;
            S.s_err = 0;
            S.s_kmax = 0;
        }
        int sp = 1;
        __syncthreads();
        while (sp > 0) {
            --sp;
            const int x = S.stk_lo[sp], y = S.stk_hi[sp];
            const int span = y - x;
            const int nslot = DENSE ? span : H + hash_pad(H);
            __syncthreads();
            // ---- clear the accumulator
            if (DENSE) {
                for (int s = tid; s < ceil_div(span, 32); s += T) S.bitmap[s] = 0u;
            } else {
                for (int s = tid; s < nslot; s += T) S.keys[s] = -1;
            }
            for (int s = tid; s < nslot; s += T) S.cnt[s] = 0;
            if (tid == 0) {
                S.s_count = 0;
                S.s_prod = 0;
                S.s_lcur = 0;
            }
            __syncthreads();
            const float scale = DENSE ? 0.f : (float)H / (float)span;

            // Streams the rows of the column's products (Algorithm 1 order), PER
            // per thread per chunk, the next chunk's loads in flight; f(u, e, row)
            // gets every product of the chunk (row -1 past the end), then
            // done() is called by all threads.
            auto expand = [&](auto &&f, auto &&done) {
                int nrow[PER];
#pragma unroll
                for (int u = 0; u < PER; ++u) nrow[u] = u * T + tid < op ? prow[u * T + tid] : -1;
                for (int e0 = 0; e0 < op; e0 += CH) {
                    int row[PER];
#pragma unroll
                    for (int u = 0; u < PER; ++u) {
                        row[u] = nrow[u];
                        const int e = e0 + CH + u * T + tid;
                        nrow[u] = e < op ? prow[e] : -1;
                    }
#pragma unroll
                    for (int u = 0; u < PER; ++u) f(u, e0 + u * T + tid, row[u]);
                    done();
                }
            };

            // A window that is the whole column and has not been split records
            // every product's slot in its destination entry during pass 1;
            // pass 2 then streams those entries instead of expanding again.
            const bool flat = W == 1 && x == lo0 && y == hi0;

            // ---- pass 1: insert rows, count products per slot
            int myfail = 0, nnew = 0, nin = 0;
            expand(
                [&](int, int e, int r) {
                    if (r < x || r >= y) return;  // also skips the padding (-1)
                    ++nin;
                    int s;
                    if (DENSE) {
                        s = r - x;
                        const unsigned bit = 1u << (s & 31);
                        const unsigned old = atomicOr(&S.bitmap[s >> 5], bit);
                        nnew += !(old & bit);
                        atomicAdd(&S.cnt[s], 1);
                    } else {
                        s = min((int)((float)(r - x) * scale), H - 1);
                        while (true) {
                            if (s >= nslot) { myfail = 1; break; }
                            int cur = S.keys[s];
                            if (cur == -1) {
                                cur = atomicCAS(&S.keys[s], -1, r);
                                if (cur == -1) {
                                    ++nnew;
                                    atomicAdd(&S.cnt[s], 1);
                                    break;
                                }
                            }
                            if (cur == r) { atomicAdd(&S.cnt[s], 1); break; }
                            ++s;
                        }
                    }
                    if (flat) a.dst[pbase + e] = (uint32_t)s;
                },
                [&]() {});
            {
                const int c = wave_sum(nnew), c2 = wave_sum(nin);
                if (lane_id() == 0 && c) atomicAdd(&S.s_count, c);
                if (lane_id() == 0 && c2) atomicAdd(&S.s_prod, c2);
            }
            const bool failed = __syncthreads_or(myfail);
            if (failed) {
                if (span <= 1 || sp + 2 > 40) {  // cannot happen: one row always fits
                    if (tid == 0) S.s_err = ERR_GROUP;
                    __syncthreads();
                    continue;
                }
                // split the window; the left half is taken first
                const int mid = x + span / 2;
                if (tid == 0) {
                    S.stk_lo[sp] = mid; S.stk_hi[sp] = y;
                    S.stk_lo[sp + 1] = x; S.stk_hi[sp + 1] = mid;
                }
                sp += 2;
                __syncthreads();
                continue;
            }

            // ---- ranks (bit 31: the slot's row is reached by several products)
            if (DENSE) {
                const int nw = ceil_div(span, 32);
                int tot;
                const int pc = tid < nw ? __builtin_popcount(S.bitmap[tid]) : 0;
                const int pre = wg_excl_scan<T>(pc, S.scan_tmp, tot);  // nw <= 128 <= T
                if (tid < nw) S.wpre[tid] = pre;
                __syncthreads();
                for (int sl = tid; sl < span; sl += T) {
                    const unsigned wd = S.bitmap[sl >> 5];
                    if ((wd >> (sl & 31)) & 1u) {
                        const int rk =
                            S.wpre[sl >> 5] + __builtin_popcount(wd & ((1u << (sl & 31)) - 1u));
                        S.rank[sl] = rk | (S.cnt[sl] > 1 ? kMulti : 0);
                    }
                }
            } else {
                // The table is ascending run by run: a row's rank is the number
                // of occupied slots before its run plus the rows of its run
                // that are smaller. Keys stay in place (pass 1 slots remain valid).
                const int per = ceil_div(nslot, T);
                const int s0 = tid * per, s1 = min(nslot, s0 + per);
                int mycnt = 0;
                for (int sl = s0; sl < s1; ++sl) mycnt += S.keys[sl] != -1;
                int tot;
                int run = wg_excl_scan<T>(mycnt, S.scan_tmp, tot);
                int cs = -1, ce = -1;  // bounds of the current run of occupied slots
                for (int sl = s0; sl < s1; ++sl) {
                    const int ks = S.keys[sl];
                    if (ks == -1) { cs = -1; continue; }
                    if (cs < 0) {
                        cs = sl;
                        while (cs > 0 && S.keys[cs - 1] != -1) --cs;
                        ce = sl + 1;
                        while (ce < nslot && S.keys[ce] != -1) ++ce;
                    }
                    int less = 0;
                    for (int t = cs; t < ce; ++t) less += S.keys[t] < ks;
                    S.rank[sl] = (run - (sl - cs) + less) | (S.cnt[sl] > 1 ? kMulti : 0);
                    ++run;
                }
            }
            // later products of this window: one reservation in the later list
            if (tid == 0 && S.s_prod > S.s_count)
                S.s_lbase = (long long)atomicAdd(&a.hdr->later_count,
                                                 (unsigned long long)(S.s_prod - S.s_count));
            __syncthreads();
            for (int sl = tid; sl < nslot; sl += T) S.cnt[sl] = 0;
            __syncthreads();

            // ---- pass 2: destinations (and the output order of a column with
            // one window and at most kSortMax products)
            const bool order_out = W == 1 && op <= kSortMax;
            int slot[PER], rk[PER];
            bool pend[PER];
            long long eg[PER];
            int myerr = 0;
            // resolves one product given its slot (or -1)
            auto settle = [&](int u, long long e, int sl) {
                slot[u] = -1;
                pend[u] = false;
                if (sl < 0) return;
                const int v = S.rank[sl];
                eg[u] = e;
                rk[u] = total + (v & 0x7fffffff);
                if (v & kMulti) {
                    slot[u] = sl;
                    pend[u] = true;
                } else {
                    a.dst[e] = (uint32_t)rk[u];
                    if (order_out) {
                        a.perm[pbase + rk[u]] = (int)(e - pbase);
                        a.crow[pbase + rk[u]] = DENSE ? x + sl : S.keys[sl];
                    }
                }
            };
            // occurrence indices of products sharing a slot, in list order
            auto order = [&]() {
                bool any = false;
#pragma unroll
                for (int u = 0; u < PER; ++u) any = any || pend[u];
                if (!__syncthreads_or(any)) return;
                if (round + CH + 1 > kRoundLimit) {  // keep rounds inside their stamp bits
                    for (int sl = tid; sl < CF::TBL; sl += T) S.stamps[sl] = 0;
                    round = 0;
                    __syncthreads();
                }
                int more;
                do {
                    ++round;
                    unsigned mine[PER];
#pragma unroll
                    for (int u = 0; u < PER; ++u) {
                        mine[u] = (round << PB) | (unsigned)(CH - 1 - (u * T + tid));
                        if (pend[u]) atomicMax(&S.stamps[slot[u]], mine[u]);
                    }
                    __syncthreads();
                    bool left = false;
#pragma unroll
                    for (int u = 0; u < PER; ++u) {
                        if (pend[u] && S.stamps[slot[u]] == mine[u]) {
                            const int k = S.cnt[slot[u]];
                            S.cnt[slot[u]] = k + 1;
                            if (k == 0) {
                                a.dst[eg[u]] = (uint32_t)rk[u];
                                if (order_out) {
                                    a.perm[pbase + rk[u]] = (int)(eg[u] - pbase);
                                    a.crow[pbase + rk[u]] =
                                        DENSE ? x + slot[u] : S.keys[slot[u]];
                                }
                            } else {
                                const long long lix = S.s_lbase + atomicAdd(&S.s_lcur, 1);
                                if (lix < a.later_cap) {
                                    a.dst[eg[u]] = kDstLater | (uint32_t)lix;
                                    a.lk[lix] = k;
                                    a.lr[lix] = rk[u];
                                    atomicMax(&S.s_kmax, k);
                                } else {
                                    myerr = ERR_GROUP;
                                }
                            }
                            pend[u] = false;
                        }
                        left = left || pend[u];
                    }
                    more = __syncthreads_or(left);
                } while (more);
            };
            if (flat) {
                // every product of the column is in this window: stream the slots
                for (int e0 = 0; e0 < op; e0 += CH) {
                    int sl[PER];
#pragma unroll
                    for (int u = 0; u < PER; ++u) {
                        const int e = e0 + u * T + tid;
                        sl[u] = e < op ? (int)a.dst[pbase + e] : -1;
                        if (sl[u] >= nslot) { myerr = ERR_GROUP; sl[u] = -1; }  // cannot happen
                    }
#pragma unroll
                    for (int u = 0; u < PER; ++u) settle(u, pbase + e0 + u * T + tid, sl[u]);
                    order();
                }
            } else {
                expand(
                    [&](int u, int e, int r) {
                        int sl = -1;
                        if (r >= x && r < y) {
                            if (DENSE) {
                                sl = r - x;
                            } else {
                                sl = min((int)((float)(r - x) * scale), H - 1);
                                while (sl < nslot && S.keys[sl] != r) ++sl;
                                if (sl >= nslot) { myerr = ERR_GROUP; sl = -1; }  // cannot happen
                            }
                        }
                        settle(u, pbase + e, sl);
                    },
                    order);
            }
            if (myerr) S.s_err = myerr;
            __syncthreads();
            total += S.s_count;
        }
        if (tid == 0) {
            if (S.s_err) atomicOr(&a.hdr->err, S.s_err);
            if (S.s_kmax) atomicMax(&a.hdr->later_maxk, S.s_kmax);
            if (!DENSE) a.itemcnt[it] = total;
            atomicAdd(&a.gnnz[g], total);
        }
        __syncthreads();
    }
}

hipError_t launch_window(const KArgs &a, int mode, int grid, hipStream_t s) {
    if (grid <= 0) return hipSuccess;
#define SPG_LAUNCH(M) hipLaunchKernelGGL((k_window<M>), dim3(grid), dim3(WinCfg<M>::T), 0, s, a)
    if (mode == WIN_DENSE) SPG_LAUNCH(WIN_DENSE);
    else if (mode == WIN_HASH_S) SPG_LAUNCH(WIN_HASH_S);
    else if (mode == WIN_HASH_L) SPG_LAUNCH(WIN_HASH_L);
    else SPG_LAUNCH(WIN_HASH_XL);
#undef SPG_LAUNCH
    return hipGetLastError();
}

}  // namespace spg
