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
//
// Products are taken in the order Algorithm 1 meets them (B entries in
// storage order, then A's rows in storage order), kBlock at a time. Products
// of one chunk that land on the same row are added in that order: every
// pending thread offers (round, thread) to the slot with an LDS atomic max,
// the lowest thread wins, adds and retires; the others retry next round. The
// values therefore match Algorithm 1 bit for bit.
//
// A window whose distinct rows overflow the table (linear probing never
// wraps; a probe running past the table's overrun area fails) is split in
// halves and each half is redone. The set of occupied slots of linear
// probing does not depend on the insertion order, so the symbolic and the
// numeric pass split identically.
#include "devutil.h"

namespace spg {

template <typename V, bool NUM, bool DENSE>
struct WinSmem {
    static constexpr int TBL = DENSE ? kDenseRows : kHashMax + kHashPad;
    int keys[DENSE ? 1 : TBL];
    unsigned bitmap[DENSE ? kDenseRows / 32 : 1];
    unsigned stamps[NUM ? TBL : 1];
    V vals[NUM ? TBL : 1];
    int s_acp[kBlock];
    int s_eoff[kBlock];
    V s_b[NUM ? kBlock : 1];
    int scan_tmp[kBlock / 64 + 1];
    int stk_lo[40], stk_hi[40];
    int s_fail, s_count, s_err;
};

template <typename V, bool NUM, bool DENSE>
__global__ __launch_bounds__(kBlock) void k_window(KArgs a) {
    using SM = WinSmem<V, NUM, DENSE>;
    __shared__ SM S;
    if (a.hdr->err) return;
    const int tid = threadIdx.x;
    const int bin = DENSE ? BIN_DENSE : BIN_HASH;
    int bstart = 0;
    for (int b = 0; b < bin; ++b) bstart += a.hdr->bin_count[b];
    const int ncolsbin = a.hdr->bin_count[bin];
    const int nitems = DENSE ? ncolsbin : a.hdr->item_count;
    if (!DENSE && nitems > a.item_cap) return;

    unsigned round = 0;
    if (NUM) {
        for (int s = tid; s < SM::TBL; s += kBlock) S.stamps[s] = 0;
        __syncthreads();
    }

    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        int g, w = 0, W = 1;
        if (DENSE) {
            g = a.binlist[bstart + it];
        } else {
            const int h = last_le(a.firstitem, ncolsbin, it);
            g = a.binlist[bstart + h];
            w = it - a.firstitem[h];
            W = a.binw[g] >> 8;
        }
        const int pid = find_prob(a, g);
        const Prob d = get_prob(a, pid);
        const int j = g - d.col0;
        const int op = a.op[g];
        const int lo0 = (int)(((long long)w * d.m) / W);
        const int hi0 = (int)(((long long)(w + 1) * d.m) / W);
        const int H = DENSE ? 0 : hash_table_size(op, W);
        const int bs = d.bcp[j], be = d.bcp[j + 1];

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
            const int nslot = DENSE ? span : H + kHashPad;
            __syncthreads();
            // ---- clear the accumulator
            if (DENSE) {
                for (int s = tid; s < ceil_div(span, 32); s += kBlock) S.bitmap[s] = 0u;
            } else {
                for (int s = tid; s < nslot; s += kBlock) S.keys[s] = -1;
            }
            if (NUM)
                for (int s = tid; s < nslot; s += kBlock) S.vals[s] = V(0);
            if (tid == 0) { S.s_fail = 0; S.s_count = 0; }
            if (NUM && round > (1u << 23)) {  // keep stamps within 24 round bits
                for (int s = tid; s < SM::TBL; s += kBlock) S.stamps[s] = 0;
                round = 0;
            }
            __syncthreads();
            const float scale = DENSE ? 0.f : (float)H / (float)span;

            bool failed = false;
            for (int bw = bs; bw < be && !failed; bw += kBlock) {
                const int t = bw + tid;
                int z = 0, acp = 0;
                V b = V(0);
                if (t < be) {
                    const int k = d.bri[t];
                    if (k >= 0 && k < d.k) {
                        acp = d.acp[k];
                        z = d.acp[k + 1] - acp;
                    }
                    if (NUM) b = ((const V *)d.bv)[t];
                }
                int Ew;
                const int ex = block_excl_scan(z, S.scan_tmp, Ew);
                S.s_acp[tid] = acp;
                S.s_eoff[tid] = ex;
                if (NUM) S.s_b[tid] = b;
                __syncthreads();
                const int nbw = min(kBlock, be - bw);
                for (int e0 = 0; e0 < Ew; e0 += kBlock) {
                    const int e = e0 + tid;
                    bool valid = e < Ew;
                    int row = -1;
                    V val = V(0);
                    if (valid) {
                        const int tt = last_le(S.s_eoff, nbw, e);
                        const int q = S.s_acp[tt] + e - S.s_eoff[tt];
                        row = d.ari[q];
                        if (NUM) val = ((const V *)d.av)[q] * S.s_b[tt];
                        if (row < 0 || row >= d.m) { S.s_err = ERR_CSC; valid = false; }
                    }
                    valid = valid && row >= x && row < y;
                    int slot = -1;
                    bool isnew = false;
                    if (valid) {
                        if (DENSE) {
                            slot = row - x;
                            const unsigned bit = 1u << (slot & 31);
                            const unsigned old = atomicOr(&S.bitmap[slot >> 5], bit);
                            isnew = !(old & bit);
                        } else {
                            int s = min((int)((float)(row - x) * scale), H - 1);
                            while (true) {
                                if (s >= nslot) { S.s_fail = 1; break; }
                                int cur = S.keys[s];
                                if (cur == -1) {
                                    cur = atomicCAS(&S.keys[s], -1, row);
                                    if (cur == -1) { isnew = true; slot = s; break; }
                                }
                                if (cur == row) { slot = s; break; }
                                ++s;
                            }
                        }
                    }
                    if (!NUM) {
                        const int c = popc64(ballot(isnew));
                        if (lane_id() == 0 && c) atomicAdd(&S.s_count, c);
                    } else {
                        // ordered accumulation: lowest thread (earliest product) first
                        bool pending = slot >= 0;
                        int more;
                        do {
                            ++round;
                            const unsigned mine = (round << 8) | (unsigned)(kBlock - 1 - tid);
                            if (pending) atomicMax(&S.stamps[slot], mine);
                            __syncthreads();
                            if (pending && S.stamps[slot] == mine) {
                                S.vals[slot] = S.vals[slot] + val;
                                pending = false;
                            }
                            more = __syncthreads_or(pending);
                        } while (more);
                    }
                    __syncthreads();
                    if (S.s_fail) { failed = true; break; }
                }
                __syncthreads();
            }
            if (failed || S.s_fail) {
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
                for (int s0 = tid; s0 < nslot; s0 += kBlock) {
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
            const int per = ceil_div(nslot, kBlock);
            const int s0 = tid * per, s1 = min(nslot, s0 + per);
            int mycnt = 0;
            for (int s = s0; s < s1; ++s) {
                const bool occ = DENSE ? ((S.bitmap[s >> 5] >> (s & 31)) & 1u) : (S.keys[s] != -1);
                mycnt += occ;
            }
            int tot;
            int pos = block_excl_scan(mycnt, S.scan_tmp, tot);
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

hipError_t launch_window(const KArgs &a, bool numeric, bool f64, bool dense, int grid,
                         hipStream_t s) {
    if (grid <= 0) return hipSuccess;
#define SPG_LAUNCH(V, N, D) \
    hipLaunchKernelGGL((k_window<V, N, D>), dim3(grid), dim3(kBlock), 0, s, a)
    if (f64) {
        if (numeric) { if (dense) SPG_LAUNCH(double, true, true); else SPG_LAUNCH(double, true, false); }
        else { if (dense) SPG_LAUNCH(double, false, true); else SPG_LAUNCH(double, false, false); }
    } else {
        if (numeric) { if (dense) SPG_LAUNCH(float, true, true); else SPG_LAUNCH(float, true, false); }
        else { if (dense) SPG_LAUNCH(float, false, true); else SPG_LAUNCH(float, false, false); }
    }
#undef SPG_LAUNCH
    return hipGetLastError();
}

}  // namespace spg
