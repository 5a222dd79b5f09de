// LDS accumulators for heavier columns, one workgroup per (column, row window):
//
//   DENSE: the SPA of Section 2.2 restricted to LDS -- a value slot per row of
//          the window plus an occupancy bitmap; rows come out ascending by
//          scanning the bitmap.
//   HASH:  the hash accumulator of Section 3.2 -- an open-addressing table with
//          linear probing, sized per column from its product count (its
//          size adaptation). The hash is order-preserving,
//          h(i) = floor((i - lo) * H / (hi - lo)), and probes never wrap, so
//          every run of occupied slots only holds rows whose home slots lie in
//          it; sorting each run in place leaves the whole table ascending.
//          Three instantiations differ only in the largest table (LDS
//          footprint) and in the workgroup size.
//
// The products of the window come from its slice of the column's product list
// (k_list.hip), already in the order Algorithm 1 meets them. They are taken
// PER * T at a time, each thread holding PER products; the loads of the next
// chunk are issued before the current chunk is accumulated. Products of one
// chunk that land on the same row are added in list order: every pending
// product offers (round, position in chunk) to its slot with an LDS atomic
// max, the earliest product wins, adds and retires; the others retry next
// round. The values therefore match Algorithm 1 bit for bit.
//
// A window whose distinct rows overflow the table (linear probing never
// wraps; a probe running past the table's overrun area fails) is split in
// halves and each half is redone from the same slice. The set of occupied
// slots of linear probing does not depend on the insertion order, so the
// symbolic and the numeric pass split identically.
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

template <typename V, bool NUM, int MODE>
struct WinSmem {
    using C = WinCfg<MODE>;
    int keys[C::DENSE ? 1 : C::TBL];
    unsigned bitmap[C::DENSE ? kDenseRows / 32 : 1];
    unsigned stamps[NUM ? C::TBL : 1];
    V vals[NUM ? C::TBL : 1];
    int scan_tmp[C::T / 64 + 1];
    int stk_lo[40], stk_hi[40];
    int s_count, s_err;
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

template <typename V, bool NUM, int MODE>
__global__ __launch_bounds__(WinCfg<MODE>::T) void k_window(KArgs a) {
    using CF = WinCfg<MODE>;
    using SM = WinSmem<V, NUM, MODE>;
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
    if (NUM) {
        for (int s = tid; s < CF::TBL; s += T) S.stamps[s] = 0;
        __syncthreads();
    }

    for (int li = blockIdx.x; li < nitems; li += gridDim.x) {
        const int it = istart + li;
        int g, w = 0, W = 1, len;
        long long lst;
        if (DENSE) {
            g = a.binlist[dstart + li].x;
            lst = a.colprod[li];  // dense columns open the list range
            len = a.op[g];
        } else {
            const int4 iw = a.items[it];
            g = iw.x;
            w = iw.y;
            W = a.binw[g] >> 8;
            lst = a.itemstart[it];
            len = a.itemlen[it];
        }
        const int pid = find_prob(a, g);
        const Prob d = get_prob(a, pid);
        const int j = g - d.col0;
        const int op = a.op[g];
        const int lo0 = window_lo(w, W, d.m);
        const int hi0 = window_lo(w + 1, W, d.m);
        const int H = DENSE ? 0 : hash_table_size(op, W);
        const int *__restrict__ lrow = a.lrow + lst;
        const int2 *__restrict__ lqp = a.lqp + lst;
        const V *__restrict__ av = (const V *)d.av;
        const V *__restrict__ bv = (const V *)d.bv;

        long long outpos = 0;
        int outlen = 0;
        if (NUM) {
            outpos = d.ccp[j];
            outlen = d.ccp[j + 1] - d.ccp[j];
            if (!DENSE)
                for (int x = 0; x < w; ++x) {
                    const int c = a.itemcnt[it - w + x];
                    outpos += c;
                    outlen -= c;
                }
        }
        int total = 0;
        if (tid == 0) {
            S.stk_lo[0] = lo0;
            S.stk_hi[0] = hi0;
            S.s_err = 0;
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
            if (NUM)
                for (int s = tid; s < nslot; s += T) S.vals[s] = V(0);
            if (tid == 0) S.s_count = 0;
            if (NUM && round > kRoundLimit) {  // keep the round inside its stamp bits
                for (int s = tid; s < CF::TBL; s += T) S.stamps[s] = 0;
                round = 0;
            }
            __syncthreads();
            const float scale = DENSE ? 0.f : (float)H / (float)span;

            int myfail = 0;
            // products of the chunk starting at c0 (loads in flight)
            int nrow[PER];
            int2 nqp[PER];
            auto fetch = [&](int c0) {
#pragma unroll
                for (int u = 0; u < PER; ++u) {
                    const int e = c0 + u * T + tid;
                    nrow[u] = -1;
                    if (e < len) {
                        nrow[u] = lrow[e];
                        if (NUM) nqp[u] = lqp[e];
                    }
                }
            };
            fetch(0);
            for (int e0 = 0; e0 < len; e0 += CH) {
                int row[PER];
                V val[PER];
#pragma unroll
                for (int u = 0; u < PER; ++u) {
                    row[u] = nrow[u];
                    if (NUM && row[u] >= 0) val[u] = av[nqp[u].x] * bv[nqp[u].y];
                }
                if (e0 + CH < len) fetch(e0 + CH);
                int slot[PER];
                int nnew = 0;
#pragma unroll
                for (int u = 0; u < PER; ++u) {
                    slot[u] = -1;
                    const int r = row[u];
                    if (r < x || r >= y) continue;  // also skips the padding (-1)
                    if (DENSE) {
                        const int sl = r - x;
                        const unsigned bit = 1u << (sl & 31);
                        const unsigned old = atomicOr(&S.bitmap[sl >> 5], bit);
                        nnew += !(old & bit);
                        slot[u] = sl;
                    } else {
                        int s = min((int)((float)(r - x) * scale), H - 1);
                        while (true) {
                            if (s >= nslot) { myfail = 1; break; }
                            int cur = S.keys[s];
                            if (cur == -1) {
                                cur = atomicCAS(&S.keys[s], -1, r);
                                if (cur == -1) { ++nnew; slot[u] = s; break; }
                            }
                            if (cur == r) { slot[u] = s; break; }
                            ++s;
                        }
                    }
                }
                if (!NUM) {
                    const int c = wave_sum(nnew);
                    if (lane_id() == 0 && c) atomicAdd(&S.s_count, c);
                } else {
                    // ordered accumulation: earliest product of each slot first
                    bool pend[PER];
#pragma unroll
                    for (int u = 0; u < PER; ++u) pend[u] = slot[u] >= 0;
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
                        bool any = false;
#pragma unroll
                        for (int u = 0; u < PER; ++u) {
                            if (pend[u] && S.stamps[slot[u]] == mine[u]) {
                                S.vals[slot[u]] = S.vals[slot[u]] + val[u];
                                pend[u] = false;
                            }
                            any = any || pend[u];
                        }
                        more = __syncthreads_or(any);
                    } while (more);
                }
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
            if (!NUM) {
                total += S.s_count;
                continue;
            }
            // ---- sort every run of occupied slots (hash only)
            if (!DENSE) {
                for (int s0 = tid; s0 < nslot; s0 += T) {
                    if (S.keys[s0] == -1 || (s0 > 0 && S.keys[s0 - 1] != -1)) continue;
                    int e = s0 + 1;
                    while (e < nslot && S.keys[e] != -1) ++e;
                    for (int u = s0 + 1; u < e; ++u) {
                        const int ku = S.keys[u];
                        const V vu = S.vals[u];
                        int v = u - 1;
                        while (v >= s0 && S.keys[v] > ku) {
                            S.keys[v + 1] = S.keys[v];
                            S.vals[v + 1] = S.vals[v];
                            --v;
                        }
                        S.keys[v + 1] = ku;
                        S.vals[v + 1] = vu;
                    }
                }
                __syncthreads();
            }
            // ---- emit occupied slots in slot order
            const int per = ceil_div(nslot, T);
            const int s0 = tid * per, s1 = min(nslot, s0 + per);
            int mycnt = 0;
            for (int s = s0; s < s1; ++s) {
                const bool occ = DENSE ? ((S.bitmap[s >> 5] >> (s & 31)) & 1u) : (S.keys[s] != -1);
                mycnt += occ;
            }
            int tot;
            int pos = wg_excl_scan<T>(mycnt, S.scan_tmp, tot);
            if (total + tot > outlen) {
                if (tid == 0) S.s_err = ERR_GROUP;
            } else {
                for (int s = s0; s < s1; ++s) {
                    const bool occ =
                        DENSE ? ((S.bitmap[s >> 5] >> (s & 31)) & 1u) : (S.keys[s] != -1);
                    if (!occ) continue;
                    const long long o = outpos + total + pos;
                    d.cri[o] = DENSE ? x + s : S.keys[s];
                    ((V *)d.cv)[o] = S.vals[s];
                    ++pos;
                }
            }
            total += tot;
            __syncthreads();
        }
        if (tid == 0) {
            if (S.s_err) atomicOr(&a.hdr->err, S.s_err);
            if (!NUM) {
                if (!DENSE) a.itemcnt[it] = total;
                atomicAdd(&a.gnnz[g], total);
            }
        }
        __syncthreads();
    }
}

hipError_t launch_window(const KArgs &a, bool numeric, bool f64, int mode, int grid,
                         hipStream_t s) {
    if (grid <= 0) return hipSuccess;
#define SPG_LAUNCH(V, N, M) \
    hipLaunchKernelGGL((k_window<V, N, M>), dim3(grid), dim3(WinCfg<M>::T), 0, s, a)
#define SPG_MODES(V, N)                                                \
    do {                                                               \
        if (mode == WIN_DENSE) SPG_LAUNCH(V, N, WIN_DENSE);            \
        else if (mode == WIN_HASH_S) SPG_LAUNCH(V, N, WIN_HASH_S);     \
        else if (mode == WIN_HASH_L) SPG_LAUNCH(V, N, WIN_HASH_L);     \
        else SPG_LAUNCH(V, N, WIN_HASH_XL);                            \
    } while (0)
    if (f64) {
        if (numeric) SPG_MODES(double, true); else SPG_MODES(double, false);
    } else {
        if (numeric) SPG_MODES(float, true); else SPG_MODES(float, false);
    }
#undef SPG_MODES
#undef SPG_LAUNCH
    return hipGetLastError();
}

}  // namespace spg
