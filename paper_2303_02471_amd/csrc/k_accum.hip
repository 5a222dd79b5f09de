// Direct-gather accumulators: expand-sort-compress (Section 4) of every output
// column, with the column's products gathered straight from A through its
// stored B entries, in two modes sharing one code path:
//   COUNT  (symbolic phase): the number of distinct rows of every column;
//   FILL   (numeric phase):  the rows in ascending order and their values,
//          each summed in Algorithm 1's order (B's stored order, starting from
//          zero, every product and sum rounded on its own), written
//          contiguously at the column's place in C.
// Nothing per product is kept between the phases.
//
// Wave buffer. A wavefront holds N = 64 KPL positions, KPL consecutive
// positions per lane (position s = KPL lane + r in register r). The columns of
// a work item occupy aligned segments of S positions; a column's products fill
// its segment in the order Algorithm 1 meets them (stored B entries in storage
// order, then the rows of the selected A column in storage order), the rest of
// the segment is padding that sorts last.
//
// Gather. A product's address in A is (start of its entry's A column) +
// (its position) - (the entry's first position). The wave writes, at the first
// position of every stored B entry, that difference and the entry's B value
// (a "head"); every other position takes the head before it (a forward fill,
// first inside each lane's registers, then across lanes by a shuffle scan).
// All of a lane's loads of A are then independent and issued together.
//
// Sort and compress. Keys (row << 11 | position) are sorted inside every
// segment by a bitonic network on registers (distances below KPL) and lanes
// (DPP, ds_swizzle, ds_bpermute). Equal rows form runs whose positions are in
// Algorithm 1's order; a run's head adds the run's values in that order.
//
// Heavy columns (more products than a wave buffer holds) are cut into row
// windows of equal span, each an independent wave work item that compacts the
// window's products (from a per-column expansion into a scratch area) into its
// buffer; a window that still overflows is halved in row span.
#include <climits>

#include "devutil.h"

namespace spg {

constexpr int kKeyBits = 11;          // position bits of a key (N <= 2048)
constexpr int kHeavyBin = BIN_SORT2;  // first bin of the heavy columns (above 1024 products)
constexpr int kHeadNone = INT_MIN;    // no head at this position

__device__ __forceinline__ void wsync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename K>
struct KeyTraits;
template <>
struct KeyTraits<unsigned> {
    static constexpr unsigned kmax = ~0u;
};
template <>
struct KeyTraits<unsigned long long> {
    static constexpr unsigned long long kmax = ~0ull;
};

// value of `v` in the lane `d` below (lanes below d read their own)
__device__ __forceinline__ int shfl_up_i(int v, int d) {
    const int l = lane_id();
    return __builtin_amdgcn_ds_bpermute((l >= d ? l - d : l) << 2, v);
}
__device__ __forceinline__ double shfl_up_v(double v, int d) {
    const unsigned long long b = __double_as_longlong(v);
    const int lo = shfl_up_i((int)(unsigned)b, d), hi = shfl_up_i((int)(unsigned)(b >> 32), d);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
__device__ __forceinline__ float shfl_up_v(float v, int d) {
    return __int_as_float(shfl_up_i(__float_as_int(v), d));
}

template <int J>
__device__ __forceinline__ unsigned kx(unsigned v) {
    return (unsigned)shfl_xor_c<J>((int)v);
}
template <int J>
__device__ __forceinline__ unsigned long long kx(unsigned long long v) {
    return shfl_xor_c64<J>(v);
}

// Median of three unsigned 32-bit values where c is 0 (the smaller of x and
// y) or all ones (the larger): one v_med3_u32 takes a compare-exchange's side
// chosen per lane.
// (Written as the instruction itself: spelled as min and max, the network's
// chains of them send the compiler's combiner into a very long search.)
__device__ __forceinline__ unsigned med3u(unsigned x, unsigned y, unsigned c) {
    unsigned r;
    asm("v_med3_u32 %0, %1, %2, %3" : "=v"(r) : "v"(x), "v"(y), "v"(c));
    return r;
}

// one compare-exchange stage between lanes at distance J (J >= 1)
template <typename K, int KPL, int J, int S>
__device__ __forceinline__ void lane_stage(K (&key)[KPL], int k, int lane) {
    const int s0 = lane * KPL;
    const bool asc = k == S || (s0 & k) == 0;
    const bool take_min = asc == ((lane & J) == 0);
    if constexpr (sizeof(K) == 4) {
        const unsigned c = take_min ? 0u : ~0u;
#pragma unroll
        for (int r = 0; r < KPL; ++r) key[r] = (K)med3u((unsigned)key[r], kx<J>((unsigned)key[r]), c);
    } else {
#pragma unroll
        for (int r = 0; r < KPL; ++r) {
            const K o = kx<J>(key[r]);
            const K mn = key[r] < o ? key[r] : o;
            const K mx = key[r] < o ? o : key[r];
            key[r] = take_min ? mn : mx;
        }
    }
}

// every aligned segment of S positions sorted ascending (bitonic network of
// the segment's size; the last merge ascending everywhere)
template <typename K, int KPL, int S>
__device__ __forceinline__ void seg_sort(K (&key)[KPL], int lane_in) {
    // The direction masks below depend on the lane only: an opaque copy of
    // the lane number keeps them from being computed once outside the
    // caller's loop and held in registers for the whole kernel.
    int lane = lane_in;
    asm volatile("" : "+v"(lane));
    const int s0 = lane * KPL;
#pragma unroll
    for (int k = 2; k <= S; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            if (j < KPL && sizeof(K) == 4 && k >= KPL && k != S) {
                // the direction depends on the lane only (r < KPL <= k):
                // each side of a pair is one median of three
                const unsigned c = (s0 & k) == 0 ? 0u : ~0u;
#pragma unroll
                for (int r = 0; r < KPL; ++r) {
                    if (r & j) continue;
                    const int rp = r | j;
                    const unsigned x = (unsigned)key[r], y = (unsigned)key[rp];
                    key[r] = (K)med3u(x, y, c);
                    key[rp] = (K)med3u(x, y, ~c);
                }
            } else if (j < KPL) {
#pragma unroll
                for (int r = 0; r < KPL; ++r) {
                    if (r & j) continue;
                    const int rp = r | j;
                    const bool asc = k == S || ((s0 + r) & k) == 0;
                    const K x = key[r], y = key[rp];
                    const bool sw = asc ? (x > y) : (x < y);
                    key[r] = sw ? y : x;
                    key[rp] = sw ? x : y;
                }
            } else {
                switch (j / KPL) {
                    case 1: lane_stage<K, KPL, 1, S>(key, k, lane); break;
                    case 2: lane_stage<K, KPL, 2, S>(key, k, lane); break;
                    case 4: lane_stage<K, KPL, 4, S>(key, k, lane); break;
                    case 8: lane_stage<K, KPL, 8, S>(key, k, lane); break;
                    case 16: lane_stage<K, KPL, 16, S>(key, k, lane); break;
                    default: lane_stage<K, KPL, 32, S>(key, k, lane); break;
                }
            }
        }
    }
}

// LDS of one wavefront: the buffer's keys (heads before the sort, sorted keys
// after it, staged output rows last) and values (B values of the heads, then
// the products' values by position, staged output values last)
template <typename K, typename V, int N, bool FILL>
struct WaveLds {
    K key[N];
    V val[FILL ? N : 1];
    int colv[64];          // per column of the item: products, then entries found
    int seg_out[64];       // per column: output entries (run count)
    int stk[2 * 48];       // window stack (heavy columns)
};

// ---------------------------------------------------------------- shared steps
// Forward fill of the heads over the lane's KPL positions and across lanes:
// qb[r] / bv[r] of every position become those of the last head at or before
// it. hq[s] = kHeadNone marks a position without a head.
template <typename V, int KPL, bool FILL>
__device__ __forceinline__ void fill_heads(int (&qb)[KPL], V (&bb)[KPL], int lane) {
    bool has = false;
    int lq = 0;
    V lb = V(0);
#pragma unroll
    for (int r = 0; r < KPL; ++r) {
        if (qb[r] != kHeadNone) {
            has = true;
            lq = qb[r];
            if (FILL) lb = bb[r];
        }
    }
    // last head of the lanes below (inclusive scan "take the later valid")
    int hv = has ? 1 : 0, sq = lq;
    V sb = lb;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int oh = shfl_up_i(hv, d), oq = shfl_up_i(sq, d);
        V ob = V(0);
        if (FILL) ob = shfl_up_v(sb, d);
        if (lane >= d && !hv && oh) {
            hv = 1;
            sq = oq;
            if (FILL) sb = ob;
        }
    }
    // exclusive: the lane below's inclusive result
    int cq = shfl_up_i(sq, 1), ch = shfl_up_i(hv, 1);
    V cb = V(0);
    if (FILL) cb = shfl_up_v(sb, 1);
    if (lane == 0) ch = 0;
    int q = ch ? cq : kHeadNone;
    V b = cb;
#pragma unroll
    for (int r = 0; r < KPL; ++r) {
        if (qb[r] != kHeadNone) {
            q = qb[r];
            if (FILL) b = bb[r];
        }
        qb[r] = q;
        if (FILL) bb[r] = b;
    }
}

// Runs of equal rows inside every aligned segment of S positions of the sorted
// keys: head flags, the run index of every head within its segment, and the
// segment's run count (valid in every lane of the segment).
template <typename K, int KPL, int S>
__device__ __forceinline__ void seg_runs(const K (&key)[KPL], bool (&head)[KPL], int (&run)[KPL],
                                         int &seg_total, int lane_in) {
    constexpr K KMAX = KeyTraits<K>::kmax;
    // opaque lane number: the permute addresses below stay inside the
    // caller's loop instead of occupying registers for the whole kernel
    int lane = lane_in;
    asm volatile("" : "+v"(lane));
    const int s0 = lane * KPL;
    // the last key of the lane below (the previous position of this lane's first)
    K prev;
    if constexpr (sizeof(K) == 4) {
        prev = (K)(unsigned)shfl_up_i((int)key[KPL - 1], 1);
    } else {
        const int lo = shfl_up_i((int)(unsigned)key[KPL - 1], 1);
        const int hi = shfl_up_i((int)(unsigned)(key[KPL - 1] >> 32), 1);
        prev = ((K)(unsigned)hi << 32) | (unsigned)lo;
    }
    int cnt = 0;
#pragma unroll
    for (int r = 0; r < KPL; ++r) {
        const int s = s0 + r;
        const K p = r == 0 ? prev : key[r - 1];
        const bool first = (s & (S - 1)) == 0;
        head[r] = key[r] != KMAX && (first || (key[r] >> kKeyBits) != (p >> kKeyBits));
        run[r] = cnt;
        cnt += head[r] ? 1 : 0;
    }
    // exclusive prefix of the lane counts inside the segment
    const int inc = wave_incl_scan(cnt);
    int base = inc - cnt;
    if constexpr (S > KPL) {
        constexpr int LPS = S / KPL;  // lanes per segment
        const int first_lane = lane & ~(LPS - 1);
        const int seg_base = __builtin_amdgcn_ds_bpermute(first_lane << 2, base);
        base -= seg_base;
        const int last_lane = first_lane + LPS - 1;
        seg_total = __builtin_amdgcn_ds_bpermute(last_lane << 2, inc) - seg_base;
    } else {
        // segments inside one lane's registers (KPL >= S): counted per segment
        seg_total = 0;  // filled by the caller from run indices
        base = 0;
    }
#pragma unroll
    for (int r = 0; r < KPL; ++r) run[r] += base;
}

// Largest occurrence index of the sorted buffer: a product's distance to the
// head of its run (its position among the products Algorithm 1 adds into the
// same entry); raised into the header's later_maxk for the plan's statistics.
template <typename K, int KPL>
__device__ __forceinline__ void note_depth(const KArgs &a, const K (&key)[KPL],
                                           const bool (&head)[KPL], int lane) {
    constexpr K KMAX = KeyTraits<K>::kmax;
    const int s0 = lane * KPL;
    int hp[KPL];
    int last = -1;
#pragma unroll
    for (int r = 0; r < KPL; ++r) {
        if (head[r]) last = s0 + r;
        hp[r] = last;
    }
    // the last head of the lanes below (head positions increase with the lane)
    int inc = last;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int o = shfl_up_i(inc, d);
        if (lane >= d) inc = max(inc, o);
    }
    int carry = shfl_up_i(inc, 1);
    if (lane == 0) carry = -1;
    int k = 0;
#pragma unroll
    for (int r = 0; r < KPL; ++r) {
        const int h = hp[r] >= 0 ? hp[r] : carry;
        if (key[r] != KMAX && h >= 0) k = max(k, s0 + r - h);
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) k = max(k, __builtin_amdgcn_ds_bpermute((lane ^ d) << 2, k));
    if (lane == 0 && k > __atomic_load_n(&a.hdr->later_maxk, __ATOMIC_RELAXED))
        atomicMax(&a.hdr->later_maxk, k);
}

// LDS slot of sorted position q when every lane stores its KPL consecutive
// positions: the position's low bits are XORed with bits of its lane, so that
// the lanes of one store (or of one step of the heads' walks) spread over the
// banks instead of sharing a few. A permutation inside each lane's KPL slots;
// with 4 positions per lane the plain layout measured no slower.
template <int KPL>
__device__ __forceinline__ int sorted_slot(int q) {
    return KPL >= 8 ? q ^ ((q >> 5) & (KPL - 1)) : q;
}

// ---------------------------------------------------------------- one work item
// A work item: G = N / S columns (global column g[cc], first stored B entry
// bs[cc], B entries nb[cc], products op[cc]), each in its aligned segment.
template <typename K, typename V, int KPL, int S, bool FILL>
__device__ __forceinline__ void item_sort_compress(const KArgs &a, const Prob &d, int pid,
                                                   WaveLds<K, V, 64 * KPL, FILL> &L,
                                                   K (&key)[KPL], int ncol, const int *gcol,
                                                   int2a ccp_lane, int lane, int &bad) {
    constexpr int N = 64 * KPL, G = N / S;
    constexpr K KMAX = KeyTraits<K>::kmax;
    seg_sort<K, KPL, S>(key, lane);
    bool head[KPL];
    int run[KPL];
    int seg_total;
    seg_runs<K, KPL, S>(key, head, run, seg_total, lane);
    if (!FILL || a.spec_fill) note_depth<K, KPL>(a, key, head, lane);
    const int s0 = lane * KPL;
    if constexpr (S <= KPL) {
        // several segments per lane: count runs per segment in registers
#pragma unroll
        for (int r = 0; r < KPL; ++r) {
            // run index inside the segment: heads before r in the same segment
            const int seg_first = r & ~(S - 1);
            int c = 0;
#pragma unroll
            for (int q = 0; q < KPL; ++q)
                if (q >= seg_first && q < r && head[q]) ++c;
            run[r] = c;
        }
    }
    // run count per column
    if constexpr (S > KPL) {
        if ((s0 & (S - 1)) == 0) L.seg_out[s0 / S] = seg_total;
    } else {
#pragma unroll
        for (int r = 0; r < KPL; r += S) {
            int c = 0;
#pragma unroll
            for (int q = 0; q < S; ++q) c += head[r + q] ? 1 : 0;
            L.seg_out[(s0 + r) / S] = c;
        }
    }
    if constexpr (!FILL) {
        wsync();
        if (lane < ncol) a.gnnz[gcol[lane]] = L.seg_out[lane];
        wsync();
        return;
    } else {
        // sorted keys to LDS (own positions), then every head adds its run
#pragma unroll
        for (int r = 0; r < KPL; ++r) L.key[sorted_slot<KPL>(s0 + r)] = key[r];
        wsync();
        // A key's position bits index the values inside its segment. Every
        // head sums its run in order and leaves the sum in its own product's
        // slot, which no other run reads.
#pragma unroll
        for (int r = 0; r < KPL; ++r) {
            if (!head[r]) continue;
            const int s = s0 + r, ss = s & ~(S - 1), send = ss + S;
            const K row = key[r] >> kKeyBits;
            const int own = ss + (int)(key[r] & (K)(S - 1));
            V acc = V(0) + L.val[own];
            for (int q = s + 1; q < send; ++q) {
                const K kq = L.key[sorted_slot<KPL>(q)];
                if (kq == KMAX || (kq >> kKeyBits) != row) break;
                acc = acc + L.val[ss + (int)(kq & (K)(S - 1))];
            }
            L.val[own] = acc;
        }
        // output start of every column; a count that differs from the
        // symbolic phase's means other inputs (nothing is written then)
        if (lane < ncol) {
            // the column's bounds in C, loaded when the item started
            const int c0 = ccp_lane.x, clen = ccp_lane.y - c0;
            L.colv[lane] = L.seg_out[lane] == clen ? c0 : -1;
            if (a.spec_fill) a.gnnz[gcol[lane]] = L.seg_out[lane];
        }
        wsync();
        // head keys staged at segment start + run index, then written out:
        // the row from the key, the sum from the slot its position bits name
#pragma unroll
        for (int r = 0; r < KPL; ++r) {
            if (!head[r]) continue;
            const int ss = (s0 + r) & ~(S - 1);
            L.key[ss + run[r]] = key[r];
        }
        wsync();
        gmem<int32_t> *cri = to_gmem(d.cri);
        gmem<V> *cv = to_gmem((V *)d.cv);
        if constexpr (G == 1) {
            // one column: 64 consecutive entries per store
            const int c0 = L.colv[0], nout = L.seg_out[0];
            if (c0 < 0) {
                bad = 1;
            } else {
                for (int i = lane; i < nout; i += 64) {
                    const K k = L.key[i];
                    cri[c0 + i] = (int32_t)(k >> kKeyBits);
                    cv[c0 + i] = L.val[(int)(k & (K)(S - 1))];
                }
            }
        } else {
            // several columns: every lane writes its own positions
#pragma unroll
            for (int r = 0; r < KPL; ++r) {
                const int s = s0 + r, cc = s / S, i = s - cc * S;
                if (cc >= ncol) continue;
                const int c0 = L.colv[cc];
                if (c0 < 0) {
                    bad = 1;
                    continue;
                }
                if (i < L.seg_out[cc]) {
                    const K k = L.key[s];
                    cri[c0 + i] = (int32_t)(k >> kKeyBits);
                    cv[c0 + i] = L.val[cc * S + (int)(k & (K)(S - 1))];
                }
            }
        }
        wsync();
    }
}

// Products of the item's columns into the wave buffer: heads from the stored B
// entries, forward fill, gathers of A's rows (and values). Returns false when
// a column's entries do not add up to its product count (inputs changed).
template <typename K, typename V, int KPL, int S, bool FILL>
__device__ __forceinline__ bool item_gather(const KArgs &a, const Prob &d,
                                            WaveLds<K, V, 64 * KPL, FILL> &L, K (&key)[KPL],
                                            int ncol, const int *bsv, const int *nbv,
                                            const int *opv, int lane) {
    constexpr int N = 64 * KPL;
    constexpr K KMAX = KeyTraits<K>::kmax;
    const int s0 = lane * KPL;
#pragma unroll
    for (int r = 0; r < KPL; ++r) L.key[s0 + r] = (K)(unsigned)kHeadNone;
    wsync();
    const int2 *__restrict__ Ep = a.E + d.ebase;
    const gmem<const V> *__restrict__ bvp = to_gmem((const V *)d.bv);
    bool ok = true;
    // the item's stored B entries, flattened column after column
    int tot_entries = 0;
    for (int cc = 0; cc < ncol; ++cc) tot_entries += nbv[cc];
    int cc_cur = 0, cc_first = 0, run = 0;  // running product count of column cc_cur
    // column of entry x and its column's first entry (columns are few: a
    // linear walk from a known column)
    auto locate = [&](int x, int c0, int f0, int &cc, int &cf) {
        cc = c0;
        cf = f0;
        while (cc < ncol - 1 && x >= cf + nbv[cc]) {
            cf += nbv[cc];
            ++cc;
        }
    };
    // entries are walked 64 at a time (a chunk may span several columns),
    // the next chunk's loads in flight while the current one is scanned
    int ncc, ncf;
    int2 ne = make_int2(0, 0);
    V nbval = V(0);
    locate(lane, 0, 0, ncc, ncf);
    if (lane < tot_entries) {
        const int t = bsv[ncc] + (lane - ncf);
        ne = Ep[t];
        if (FILL) nbval = bvp[t];
    }
    for (int x0 = 0; x0 < tot_entries; x0 += 64) {
        const int x = x0 + lane;
        const int cc = ncc, cf = ncf;
        const int z = x < tot_entries ? ne.y : 0, as = ne.x;
        const V bval = nbval;
        if (x0 + 64 < tot_entries) {
            locate(x + 64, cc, cf, ncc, ncf);
            if (x + 64 < tot_entries) {
                const int t = bsv[ncc] + (x + 64 - ncf);
                ne = Ep[t];
                if (FILL) nbval = bvp[t];
            }
        }
        // position inside the column: exclusive prefix of z over the column's
        // entries (scan over the chunk, restarted at every column start)
        const bool seg_head = x < tot_entries && (x == cf || x == x0);
        // segmented inclusive scan: add the value of the lane below while no
        // segment head lies between
        int inc = z;
        bool blocked = seg_head;
#pragma unroll
        for (int dd = 1; dd < 64; dd <<= 1) {
            const int oi = shfl_up_i(inc, dd);
            const int ob = shfl_up_i(blocked ? 1 : 0, dd);
            if (lane >= dd && !blocked) inc += oi;
            if (lane >= dd && !blocked) blocked = ob != 0;
        }
        // carry into the chunk: the running count of the column the chunk
        // starts in, for entries of that column
        const int carry = (cc == cc_cur) ? run : 0;
        const int o = carry + inc - z;
        // the last entry of a column closes it at exactly its product count
        if (x < tot_entries && x == cf + nbv[cc] - 1 && o + z != opv[cc]) ok = false;
        if (x < tot_entries && z > 0) {
            if (o < 0 || o + z > opv[cc]) {
                ok = false;
            } else {
                L.key[cc * S + o] = (K)(unsigned)(as - o);
                if (FILL) L.val[cc * S + o] = bval;
            }
        }
        // advance: the column and running count after the chunk's last entry
        const int last = min(63, tot_entries - 1 - x0);
        const int cc_last = __builtin_amdgcn_ds_bpermute(last << 2, cc);
        const int cf_last = __builtin_amdgcn_ds_bpermute(last << 2, cf);
        const int o_last = __builtin_amdgcn_ds_bpermute(last << 2, o + z);
        cc_cur = cc_last;
        cc_first = cf_last;
        run = o_last;
    }
    ok = __builtin_amdgcn_ballot_w64(!ok) == 0;
    wsync();
    int qb[KPL];
    V bb[KPL];
#pragma unroll
    for (int r = 0; r < KPL; ++r) {
        qb[r] = (int)(unsigned)L.key[s0 + r];
        bb[r] = FILL ? L.val[s0 + r] : V(0);
    }
    fill_heads<V, KPL, FILL>(qb, bb, lane);
    // The filled heads go back to LDS by position, and the gathers take
    // positions lane-major (position 64 r + lane in register r): consecutive
    // lanes then read consecutive entries of the same A column, so a load
    // instruction touches a few cache lines instead of up to 64.
#pragma unroll
    for (int r = 0; r < KPL; ++r) {
        L.key[s0 + r] = (K)(unsigned)qb[r];
        if (FILL) L.val[s0 + r] = bb[r];
    }
    wsync();
    const gmem<const int32_t> *__restrict__ ari = to_gmem(d.ari);
    const gmem<const V> *__restrict__ av = to_gmem((const V *)d.av);
    int row[KPL];
    bool live[KPL];
    V x[KPL];
    // every gather of the lane issued before any is used (the B value of
    // each position stays in LDS until its product replaces it)
#pragma unroll
    for (int r = 0; r < KPL; ++r) {
        const int s = r * 64 + lane, cc = s / S, i = s & (S - 1);
        const int qs = (int)(unsigned)L.key[s];
        live[r] = ok && cc < ncol && i < opv[cc] && qs != kHeadNone;
        const int q = live[r] ? qs + i : 0;
        row[r] = live[r] ? ari[q] : 0;
        if (FILL) x[r] = live[r] ? av[q] : V(0);
    }
    wsync();  // every lane has read the filled heads
    bool badrow = false;
#pragma unroll
    for (int r = 0; r < KPL; ++r) {
        const int s = r * 64 + lane, i = s & (S - 1);
        // a row outside A's row range is malformed input (reported; the
        // product takes no part)
        if (live[r] && (row[r] < 0 || row[r] >= d.m)) {
            badrow = true;
            live[r] = false;
        }
        L.key[s] = live[r] ? (((K)(unsigned)row[r] << kKeyBits) | (K)(unsigned)i) : KMAX;
        if (FILL && live[r]) L.val[s] = x[r] * L.val[s];
    }
    if (ballot(badrow) && lane == 0) atomicOr(&a.hdr->err, ERR_CSC);
    wsync();
    // keys back in the sort's layout: positions s0 .. s0 + KPL - 1 per lane;
    // a buffer that is one segment may start the sort in any order, so its
    // lanes read position 64 r + lane (consecutive lanes, consecutive banks)
#pragma unroll
    for (int r = 0; r < KPL; ++r) key[r] = L.key[S == N ? r * 64 + lane : s0 + r];
    wsync();
    return ok;
}

// ---------------------------------------------------------------- wavefront groups
// Bin `bin` holds columns of at most S products; G = N / S of them per wave.
// One wavefront per workgroup: waves share nothing.
template <typename K, typename V, int KPL, int S, bool FILL>
// The groups of 32 to 128 products are held to 96 VGPRs, 5 waves per SIMD
// instead of 4 (at the cost of 8 bytes of scratch), which measured 1.5 to 3 us
// faster each; the groups of 16 lose more to the spill than they gain.
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(KPL == 4 && S >= 32 && S < 256 ? 5 : 1))) void k_acc_wave(KArgs a, int bin) {
    constexpr int N = 64 * KPL, G = N / S;
    static_assert(S <= N && (N % S) == 0 && N <= (1 << kKeyBits), "segments tile the buffer");
    __shared__ WaveLds<K, V, N, FILL> L;
    if (__atomic_load_n(&a.hdr->err, __ATOMIC_RELAXED) |
        (FILL ? __atomic_load_n(&a.hdr->cap_over, __ATOMIC_RELAXED) : 0))
        return;
    const int lane = threadIdx.x;
    int start = 0;
    for (int b = 0; b < bin; ++b) start += a.hdr->bin_count[b];
    const int cnt = a.hdr->bin_count[bin];
    const int ngroups = ceil_div(cnt, G);
    int bad = 0;
    __shared__ int s_g[G > 64 ? 64 : G], s_bs[G > 64 ? 64 : G], s_nb[G > 64 ? 64 : G],
        s_op[G > 64 ? 64 : G];
    for (int gi = blockIdx.x; gi < ngroups; gi += gridDim.x) {
        const int first = start + gi * G, ncol = min(G, cnt - gi * G);
        if (lane < ncol) {
            const int4 ent = a.binlist[first + lane];
            s_g[lane] = ent.x;
            s_bs[lane] = ent.y;
            s_nb[lane] = ent.z;
            s_op[lane] = ent.w;
            if (ent.w > S) bad = 1;  // cannot happen for unchanged inputs
        }
        wsync();
        if (__builtin_amdgcn_ballot_w64(bad != 0)) break;
        // every column of a group belongs to one problem (bins are filled per
        // problem tile, but a group may cross problems): split by problem
        int c0 = 0;
        while (c0 < ncol) {
            const int pid = find_prob(a, s_g[c0]);
            const Prob d = get_prob(a, pid);
            int c1 = c0 + 1;
            while (c1 < ncol && s_g[c1] >= d.col0 && s_g[c1] < d.col0 + d.n) ++c1;
            K key[KPL];
            // the filling pass's column bounds in C (known before the kernel)
            // load now; they are used after the sort
            int2a ccp_lane = {0, 0};
            if (FILL && lane < c1 - c0) ccp_lane = load_pair(d.ccp, s_g[c0 + lane] - d.col0);
            if (c0 == 0 && c1 == ncol) {
                if (!item_gather<K, V, KPL, S, FILL>(a, d, L, key, ncol, s_bs, s_nb, s_op, lane))
                    bad = 1;
                else
                    item_sort_compress<K, V, KPL, S, FILL>(a, d, pid, L, key, ncol, s_g, ccp_lane,
                                                           lane, bad);
            } else {
                // a group spanning problems: each problem's columns as an item
                // of their own (at the front of the buffer)
                if (!item_gather<K, V, KPL, S, FILL>(a, d, L, key, c1 - c0, s_bs + c0, s_nb + c0,
                                                     s_op + c0, lane))
                    bad = 1;
                else
                    item_sort_compress<K, V, KPL, S, FILL>(a, d, pid, L, key, c1 - c0, s_g + c0,
                                                           ccp_lane, lane, bad);
            }
            c0 = c1;
        }
        wsync();
    }
    // an output count other than the planned one: other inputs, or (a
    // numeric phase run at a previous structure's positions) a redo
    if (__builtin_amdgcn_ballot_w64(bad != 0) && lane == 0)
        atomicOr(&a.hdr->err, a.spec_fill ? ERR_RETRY : ERR_GROUP);
}

// ---------------------------------------------------------------- one column per lane
// Columns of at most L products and L stored B entries: every lane takes one
// column whole, in its own registers -- the paper's mapping of one column to
// one vector element (Section 3.1), with a sort-merge in place of its
// accumulator. No lane talks to another; each lane's values sit in its own
// LDS slots. Keys (row << LB | position) are 32-bit while rows stay below
// 2^(32 - LB) - 1.
template <typename K, typename V, int L, bool FILL>
__global__ __launch_bounds__(64) void k_acc_lane(KArgs a, int bin) {
    constexpr int LB = L <= 4 ? 2 : (L <= 8 ? 3 : 4);
    static_assert((1 << LB) == L, "L is 4, 8 or 16");
    constexpr K KMAX = KeyTraits<K>::kmax;
    __shared__ V sval[FILL ? 64 * L : 1];
    if (__atomic_load_n(&a.hdr->err, __ATOMIC_RELAXED) |
        (FILL ? __atomic_load_n(&a.hdr->cap_over, __ATOMIC_RELAXED) : 0))
        return;
    const int lane = threadIdx.x;
    int start = 0;
    for (int b = 0; b < bin; ++b) start += a.hdr->bin_count[b];
    const int cnt = a.hdr->bin_count[bin];
    int bad = 0, badrow = 0, kmax = 0;
    for (int ci = blockIdx.x * 64 + lane; ci < cnt; ci += gridDim.x * 64) {
        const int4 ent = a.binlist[start + ci];
        const int g = ent.x, bs = ent.y, nb = ent.z, op = ent.w;
        if (op > L || nb > L) {  // cannot happen for unchanged inputs
            bad = 1;
            continue;
        }
        const int pid = find_prob(a, g);
        const Prob d = get_prob(a, pid);
        // the C column's bounds (numeric phase) load together with the entries
        int c0 = 0, clen = 0;
        if (FILL) {
            const int j = g - d.col0;
            const int2a cp = load_pair(d.ccp, j);
            c0 = cp.x;
            clen = cp.y - c0;
        }
        const int2 *__restrict__ Ep = a.E + d.ebase;
        const gmem<const V> *__restrict__ bvp = to_gmem((const V *)d.bv);
        // the column's stored B entries: A column start, length, B value
        int as_[L], zs[L], oo[L];
        V bv_[L];
#pragma unroll
        for (int t = 0; t < L; ++t) {
            as_[t] = 0;
            zs[t] = 0;
            bv_[t] = V(0);
            if (t < nb) {
                const int2 e = Ep[bs + t];
                as_[t] = e.x;
                zs[t] = e.y;
                if (FILL) bv_[t] = bvp[bs + t];
            }
        }
        int run = 0;
#pragma unroll
        for (int t = 0; t < L; ++t) {
            oo[t] = run;
            run += zs[t];
        }
        if (run != op) {  // entries do not add up to the product count
            bad = 1;
            continue;
        }
        // product p belongs to the entry after the ones ending at or before p
        int q[L];
        V bb[L];
#pragma unroll
        for (int p = 0; p < L; ++p) {
            int tp = 0;
#pragma unroll
            for (int t = 0; t < L; ++t) tp += (oo[t] + zs[t] <= p) ? 1 : 0;
            int qa = 0, qo = 0;
            V qv = V(0);
#pragma unroll
            for (int t = 0; t < L; ++t) {
                if (t == tp) {
                    qa = as_[t];
                    qo = oo[t];
                    if (FILL) qv = bv_[t];
                }
            }
            q[p] = qa + p - qo;
            bb[p] = qv;
        }
        const gmem<const int32_t> *__restrict__ ari = to_gmem(d.ari);
        const gmem<const V> *__restrict__ av = to_gmem((const V *)d.av);
        int row[L];
        V x[L];
#pragma unroll
        for (int p = 0; p < L; ++p) {
            row[p] = p < op ? ari[q[p]] : 0;
            if (FILL) x[p] = p < op ? av[q[p]] : V(0);
        }
        K key[L];
#pragma unroll
        for (int p = 0; p < L; ++p) {
            key[p] = KMAX;
            if (p < op) {
                if (row[p] < 0 || row[p] >= d.m) {
                    badrow = 1;
                } else {
                    key[p] = ((K)(unsigned)row[p] << LB) | (K)(unsigned)p;
                    if (FILL) sval[lane * L + p] = x[p] * bb[p];
                }
            }
        }
        // bitonic network over the lane's L keys
#pragma unroll
        for (int k = 2; k <= L; k <<= 1) {
#pragma unroll
            for (int jj = k >> 1; jj > 0; jj >>= 1) {
#pragma unroll
                for (int r = 0; r < L; ++r) {
                    if (r & jj) continue;
                    const int rp = r | jj;
                    const bool asc = (r & k) == 0;
                    const K u = key[r], w = key[rp];
                    const bool sw = asc ? (u > w) : (u < w);
                    key[r] = sw ? w : u;
                    key[rp] = sw ? u : w;
                }
            }
        }
        // runs of equal rows, each summed in position order (Algorithm 1's)
        int nd = 0, depth = 0, dcur = 0;
#pragma unroll
        for (int p = 0; p < L; ++p) {
            if (key[p] == KMAX) continue;
            const bool head = p == 0 || (key[p] >> LB) != (key[p - 1] >> LB);
            dcur = head ? 0 : dcur + 1;
            depth = max(depth, dcur);
            nd += head ? 1 : 0;
        }
        kmax = max(kmax, depth);
        if (!FILL || a.spec_fill) a.gnnz[g] = nd;
        if (FILL) {
            if (nd != clen) {
                bad = 1;
                continue;
            }
            gmem<int32_t> *cri = to_gmem(d.cri);
            gmem<V> *cv = to_gmem((V *)d.cv);
            int u = 0;
            V acc = V(0);
#pragma unroll
            for (int p = 0; p < L; ++p) {
                if (key[p] == KMAX) continue;
                const V v = sval[lane * L + (int)(key[p] & (K)(L - 1))];
                const bool head = p == 0 || (key[p] >> LB) != (key[p - 1] >> LB);
                acc = head ? V(0) + v : acc + v;
                const bool last = p == L - 1 || key[p + 1 < L ? p + 1 : p] == KMAX ||
                                  (key[p + 1 < L ? p + 1 : p] >> LB) != (key[p] >> LB);
                if (last) {
                    cri[c0 + u] = (int32_t)(key[p] >> LB);
                    cv[c0 + u] = acc;
                    ++u;
                }
            }
        }
    }
    if (ballot(badrow) && lane == 0) atomicOr(&a.hdr->err, ERR_CSC);
    if (ballot(bad != 0) && lane == 0)
        atomicOr(&a.hdr->err, FILL && a.spec_fill ? ERR_RETRY : ERR_GROUP);
    if (!FILL || a.spec_fill) {
#pragma unroll
        for (int dd = 32; dd >= 1; dd >>= 1)
            kmax = max(kmax, __builtin_amdgcn_ds_bpermute((lane ^ dd) << 2, kmax));
        if (lane == 0 && kmax > __atomic_load_n(&a.hdr->later_maxk, __ATOMIC_RELAXED))
            atomicMax(&a.hdr->later_maxk, kmax);
    }
}

// ---------------------------------------------------------------- heavy columns
// Plan of the heavy columns (bins SORT2, SORT3 and WSORT: more than 1024
// products; contiguous in the bin list): per column its first product in the heavy scratch (hoff) and its
// first window (wbase), W = ceil(Op / kWinTarget) windows of equal row span;
// in a planned launch also the map of windows to columns.
// One workgroup; the totals go to the header (the host sizes the scratch from
// them). A planned launch whose scratch is too small is redone.
constexpr int kWinKpl = 16;                     // positions per lane of a window's buffer
// planned products per window: 15/16 of the buffer (measured: 7/8 leaves more
// windows and rescans, 1000 of 1024 more windows that overflow and are halved)
constexpr int kWinTarget = 64 * kWinKpl * 15 / 16;

__global__ __launch_bounds__(1024) void k_heavy_plan(KArgs a) {
    constexpr int T = 1024, PT = 4;
    __shared__ int tmp[T / 64 + 1];
    __shared__ long long s_tmp[T / 64 + 1];
    if (__syncthreads_or(__atomic_load_n(&a.hdr->err, __ATOMIC_RELAXED) != 0)) return;
    int first = 0;
    for (int b = 0; b < kHeavyBin; ++b) first += a.hdr->bin_count[b];
    int n = 0;
    for (int b = kHeavyBin; b <= BIN_WSORT; ++b) n += a.hdr->bin_count[b];
    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
    long long pcarry = 0;
    int wcarry = 0;
    // PT consecutive columns per thread: one scan step covers T PT columns
    for (int i0 = 0; i0 < n; i0 += T * PT) {
        const int ib = i0 + tid * PT;
        int op[PT], nw[PT];
        int wsum = 0;
        long long v = 0;
#pragma unroll
        for (int u = 0; u < PT; ++u) {
            const int i = ib + u;
            op[u] = i < n ? a.binlist[first + i].w : 0;
            nw[u] = i < n ? max(1, ceil_div(op[u], kWinTarget)) : 0;
            wsum += nw[u];
            v += op[u];
        }
        int wt;
        const int wex = wg_excl_scan<T>(wsum, tmp, wt);
        // 64-bit prefix of the products
        long long inc = v;
#pragma unroll
        for (int dd = 1; dd < 64; dd <<= 1) {
            const int lo = shfl_up_i((int)(unsigned)inc, dd);
            const int hi = shfl_up_i((int)(unsigned)((unsigned long long)inc >> 32), dd);
            const long long o = (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
            if (l >= dd) inc += o;
        }
        if (l == 63) s_tmp[w] = inc;
        __syncthreads();
        if (tid == 0) {
            long long run = 0;
            for (int q = 0; q < T / 64; ++q) {
                const long long x = s_tmp[q];
                s_tmp[q] = run;
                run += x;
            }
            s_tmp[T / 64] = run;
        }
        __syncthreads();
        long long pr = pcarry + s_tmp[w] + inc - v;
        int wr = wcarry + wex;
#pragma unroll
        for (int u = 0; u < PT; ++u) {
            const int i = ib + u;
            if (i < n) {
                a.hoff[i] = pr;
                a.wbase[i] = wr;
                // a planned launch has its window scratch already: the
                // column's windows are mapped here (as far as it holds them;
                // more windows than it holds ask for a redo below)
                if (a.spec_total >= 0)
                    for (int q = wr; q < wr + nw[u] && q < a.win_cap; ++q) a.winmap[q] = i;
            }
            pr += op[u];
            wr += nw[u];
        }
        pcarry += s_tmp[T / 64];
        wcarry += wt;
        __syncthreads();
    }
    if (tid == 0) {
        a.hoff[n] = pcarry;
        a.wbase[n] = wcarry;
        a.hdr->heavy_prod = (unsigned long long)pcarry;
        a.hdr->heavy_win = wcarry;
        if (a.spec_total >= 0 && (pcarry > a.heavy_cap || wcarry > a.win_cap))
            atomicOr(&a.hdr->err, ERR_RETRY);
    }
}

// The heavy column of every window (one thread per heavy column), written
// once the window scratch is in place; a launch planned with too small a
// scratch has been flagged for a redo and writes nothing.
__global__ __launch_bounds__(kBlock) void k_win_map(KArgs a) {
    if (__atomic_load_n(&a.hdr->err, __ATOMIC_RELAXED)) return;
    int n = 0;
    for (int b = kHeavyBin; b <= BIN_WSORT; ++b) n += a.hdr->bin_count[b];
    for (int li = blockIdx.x * kBlock + threadIdx.x; li < n; li += gridDim.x * kBlock) {
        const int w0 = a.wbase[li], w1 = a.wbase[li + 1];
        for (int w = w0; w < w1 && w < a.win_cap; ++w) a.winmap[w] = li;
    }
}

// Expansion of the heavy columns into the scratch: the row (and in FILL the
// value A(i,k) B(k,j)) of every product, in Algorithm 1's order. One workgroup
// per heavy column (grid-stride), its stored B entries 256 at a time.
template <typename V, bool FILL>
__global__ __launch_bounds__(kBlock) void k_heavy_expand(KArgs a) {
    __shared__ int s_acp[kBlock], s_eoff[kBlock], scan_tmp[kBlock / 64 + 1];
    __shared__ V s_bv[FILL ? kBlock : 1];
    if (__syncthreads_or((__atomic_load_n(&a.hdr->err, __ATOMIC_RELAXED) |
                          (FILL ? __atomic_load_n(&a.hdr->cap_over, __ATOMIC_RELAXED) : 0)) != 0))
        return;
    int first = 0;
    for (int b = 0; b < kHeavyBin; ++b) first += a.hdr->bin_count[b];
    int n = 0;
    for (int b = kHeavyBin; b <= BIN_WSORT; ++b) n += a.hdr->bin_count[b];
    const int tid = threadIdx.x;
    int bad = 0, rowbad = 0;
    // largest columns first (the heavy list runs from small to large bins):
    // the longest workgroups start before the short ones
    for (int lj = blockIdx.x; lj < n; lj += gridDim.x) {
        const int li = n - 1 - lj;
        const int4 ent = a.binlist[first + li];
        const int g = ent.x, bs = ent.y, nb = ent.z;
        const int pid = find_prob(a, g);
        const Prob d = get_prob(a, pid);
        const long long base0 = a.hoff[li], end = a.hoff[li + 1];
        const int2 *__restrict__ Ep = a.E + d.ebase;
        const gmem<const int32_t> *__restrict__ ari = to_gmem(d.ari);
        const gmem<const V> *__restrict__ av = to_gmem((const V *)d.av);
        const gmem<const V> *__restrict__ bvp = to_gmem((const V *)d.bv);
        long long base = base0;
        for (int bw = 0; bw < nb; bw += kBlock) {
            const int t = bw + tid;
            int z = 0, as = 0;
            V bval = V(0);
            if (t < nb) {
                const int2 e = Ep[bs + t];
                as = e.x;
                z = e.y;
                if (FILL) bval = bvp[bs + t];
            }
            int Ew;
            const int ex = block_excl_scan(z, scan_tmp, Ew);
            s_acp[tid] = as;
            s_eoff[tid] = ex;
            if (FILL) s_bv[tid] = bval;
            __syncthreads();
            const int nbw = min(kBlock, nb - bw);
            if (base + Ew > end) {  // more products than planned: inputs changed
                bad = 1;
                __syncthreads();
                break;
            }
            for (int e0 = 0; e0 < Ew; e0 += 4 * kBlock) {
                int rr[4];
                V xv[4];
                int tt[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int e = e0 + u * kBlock + tid;
                    const int ee = min(e, Ew - 1);
                    tt[u] = last_le(s_eoff, nbw, ee);
                    const int q = s_acp[tt[u]] + ee - s_eoff[tt[u]];
                    rr[u] = ari[q];
                    if (FILL) xv[u] = av[q];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int e = e0 + u * kBlock + tid;
                    if (e >= Ew) continue;
                    if (rr[u] < 0 || rr[u] >= d.m) {  // malformed input
                        rowbad = 1;
                        rr[u] = 0;
                    }
                    a.hrow[base + e] = rr[u];
                    if (FILL) ((V *)a.hval)[base + e] = xv[u] * s_bv[tt[u]];
                }
            }
            base += Ew;
            __syncthreads();
        }
    }
    if (bad && tid == 0) atomicOr(&a.hdr->err, ERR_GROUP);
    if (rowbad) atomicOr(&a.hdr->err, ERR_CSC);
}

// A product index kept in a value slot of the wave buffer (its first 4 bytes)
// until the value replaces it.
template <typename V>
__device__ __forceinline__ void put_index(V &slot, int e) {
    __builtin_memcpy(&slot, &e, 4);
}
template <typename V>
__device__ __forceinline__ int get_index(const V &slot) {
    int e;
    __builtin_memcpy(&e, &slot, 4);
    return e;
}

// One window of a heavy column per wavefront (grid-stride over all windows):
// rows [m w / W, m (w + 1) / W) of the column's products, compacted in product
// order into the buffer, sorted, compressed. A window holding more products
// than the buffer is halved in row span (a stack, left half first); a window
// of a single row with more products than the buffer is one output entry,
// summed in product order by one lane.
template <typename K, typename V, bool FILL>
__global__ __launch_bounds__(64) void k_acc_window(KArgs a) {
    constexpr int KPL = kWinKpl, N = 64 * KPL;
    constexpr K KMAX = KeyTraits<K>::kmax;
    // Values gathered after the scan (one batch, one memory round trip per
    // scan step fewer) where the registers it takes cost no occupancy: 32-bit
    // keys with 8-byte values, whose wave buffer already allows 3 waves per SIMD
    constexpr bool kDefer = sizeof(K) == 4 && sizeof(V) == 8;
    __shared__ WaveLds<K, V, N, FILL> L;
    if (__atomic_load_n(&a.hdr->err, __ATOMIC_RELAXED) |
        (FILL ? __atomic_load_n(&a.hdr->cap_over, __ATOMIC_RELAXED) : 0))
        return;
    const int lane = threadIdx.x;
    int first = 0;
    for (int b = 0; b < kHeavyBin; ++b) first += a.hdr->bin_count[b];
    int n = 0;
    for (int b = kHeavyBin; b <= BIN_WSORT; ++b) n += a.hdr->bin_count[b];
    const int nwin = a.wbase[n];
    int bad = 0;
    // windows of the largest columns (the longest scans) first; workgroups go
    // to the 8 XCDs in turn and each XCD has its own L2, so every run of kRun
    // consecutive windows (mostly one column's, which all scan that column)
    // goes to one XCD: inside each block of kXcd kRun workgroups, XCD x takes
    // windows kRun x .. kRun x + kRun - 1 of the block (the ragged last block
    // keeps its order)
    constexpr int kXcd = 8, kRun = 16, kBlk = kXcd * kRun;
    const int full = nwin / kBlk * kBlk;
    for (int b = blockIdx.x; b < nwin; b += gridDim.x) {
        const int rb = b % kBlk;
        const int wj = b >= full ? b : b - rb + (rb % kXcd) * kRun + rb / kXcd;
        const int wi = nwin - 1 - wj;
        const int li = a.winmap[wi];
        const int wb = a.wbase[li], w = wi - wb, W = a.wbase[li + 1] - wb;
        const int g = a.binlist[first + li].x;
        const int pid = find_prob(a, g);
        const Prob d = get_prob(a, pid);
        const int j = g - d.col0;
        const long long hb = a.hoff[li];
        const int op = (int)(a.hoff[li + 1] - hb);
        const int *__restrict__ prow = a.hrow + hb;
        const V *__restrict__ pval = FILL ? (const V *)a.hval + hb : nullptr;
        // output position of the window: the entries of the earlier windows
        int out = 0;
        if (FILL) {
            for (int q = lane; q < w; q += 64) out += a.wcnt[wb + q];
            out = wave_sum(out);
        }
        int c0 = 0;
        if (FILL) c0 = d.ccp[j];
        const int m = d.m;
        int sp = 0;
        if (lane == 0) {
            L.stk[0] = (int)((long long)m * w / W);
            L.stk[1] = (int)((long long)m * (w + 1) / W);
        }
        sp = 1;
        wsync();
        int total = 0;
        while (sp > 0) {
            --sp;
            const int x = L.stk[2 * sp], y = L.stk[2 * sp + 1];
            wsync();
            // compact the window's products (product order) into the buffer,
            // 8 rows per lane loaded before any is tested
            constexpr int U = 8;
            int cnt = 0;
            for (int e0 = 0; e0 < op; e0 += 64 * U) {
                int r[U], pos[U];
                bool in[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int e = e0 + u * 64 + lane;
                    r[u] = e < op ? prow[e] : -1;
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    in[u] = r[u] >= x && r[u] < y;
                    const unsigned long long bm = ballot(in[u]);
                    pos[u] = cnt + popc64(bm & mask_lt());
                    cnt += popc64(bm);
                }
                // deferred: the value slot holds the product's index until
                // the scan ends; else the values are gathered here
                V vv[kDefer ? 1 : U];
                if constexpr (FILL && !kDefer) {
#pragma unroll
                    for (int u = 0; u < U; ++u)
                        vv[u] = in[u] && pos[u] < N ? pval[e0 + u * 64 + lane] : V(0);
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    if (in[u] && pos[u] < N) {
                        L.key[pos[u]] = ((K)(unsigned)r[u] << kKeyBits) | (K)(unsigned)pos[u];
                        if constexpr (FILL && kDefer) put_index(L.val[pos[u]], e0 + u * 64 + lane);
                        if constexpr (FILL && !kDefer) L.val[pos[u]] = vv[u];
                    }
                }
            }
            wsync();
            if (cnt > N && y - x > 1) {
                if (sp + 2 > 48) {  // cannot happen: the span halves every time
                    bad = 1;
                    break;
                }
                const int mid = x + (y - x) / 2;
                if (lane == 0) {
                    L.stk[2 * sp] = mid;
                    L.stk[2 * sp + 1] = y;
                    L.stk[2 * sp + 2] = x;
                    L.stk[2 * sp + 3] = mid;
                }
                sp += 2;
                wsync();
                continue;
            }
            if (cnt > N) {
                // one row, more products than the buffer: one entry
                if ((!FILL || a.spec_fill) && lane == 0 &&
                    cnt - 1 > __atomic_load_n(&a.hdr->later_maxk, __ATOMIC_RELAXED))
                    atomicMax(&a.hdr->later_maxk, cnt - 1);
                if (FILL && lane == 0) {
                    V acc = V(0);
                    bool firstp = true;
                    for (int e = 0; e < op; ++e) {
                        if (prow[e] != x) continue;
                        acc = firstp ? V(0) + pval[e] : acc + pval[e];
                        firstp = false;
                    }
                    if (out + total >= d.ccp[j + 1] - c0) bad = 1;
                    else {
                        d.cri[c0 + out + total] = x;
                        ((V *)d.cv)[c0 + out + total] = acc;
                    }
                }
                total += 1;
                wsync();
                continue;
            }
            if constexpr (FILL && kDefer) {
                // the values of the window's products, one batch of gathers
                // (the scan above waited on its rows only)
                constexpr int H = KPL / 2;  // half the slots per batch (registers)
#pragma unroll
                for (int h = 0; h < KPL; h += H) {
                    V vv[H];
#pragma unroll
                    for (int r = 0; r < H; ++r) {
                        const int s = (h + r) * 64 + lane;
                        vv[r] = s < cnt ? pval[get_index(L.val[s])] : V(0);
                    }
#pragma unroll
                    for (int r = 0; r < H; ++r) {
                        const int s = (h + r) * 64 + lane;
                        if (s < cnt) L.val[s] = vv[r];
                    }
                    wsync();
                }
            }
            // sort and compress the buffer as one segment
            K key[KPL];
            const int s0 = lane * KPL;
#pragma unroll
            for (int r = 0; r < KPL; ++r) {
                // any start order sorts the same: position 64 r + lane, so
                // that consecutive lanes read consecutive banks
                const int s = r * 64 + lane;
                key[r] = s < cnt ? L.key[s] : KMAX;
            }
            wsync();
            seg_sort<K, KPL, N>(key, lane);
            bool head[KPL];
            int run[KPL];
            int runs;
            seg_runs<K, KPL, N>(key, head, run, runs, lane);
            if (!FILL || a.spec_fill) note_depth<K, KPL>(a, key, head, lane);
            if (FILL) {
#pragma unroll
                for (int r = 0; r < KPL; ++r) L.key[sorted_slot<KPL>(s0 + r)] = key[r];
                wsync();
                // every head sums its run in order into its own product's
                // slot, then its key is staged at its run index
#pragma unroll
                for (int r = 0; r < KPL; ++r) {
                    if (!head[r]) continue;
                    const K row = key[r] >> kKeyBits;
                    const int own = (int)(key[r] & (K)(N - 1));
                    V acc = V(0) + L.val[own];
                    for (int q = s0 + r + 1; q < N; ++q) {
                        const K kq = L.key[sorted_slot<KPL>(q)];
                        if (kq == KMAX || (kq >> kKeyBits) != row) break;
                        acc = acc + L.val[(int)(kq & (K)(N - 1))];
                    }
                    L.val[own] = acc;
                }
                wsync();
#pragma unroll
                for (int r = 0; r < KPL; ++r)
                    if (head[r]) L.key[run[r]] = key[r];
                wsync();
                const int clen = d.ccp[j + 1] - c0;
                if (out + total + runs > clen) {
                    bad = 1;
                } else {
                    gmem<int32_t> *cri = to_gmem(d.cri);
                    gmem<V> *cv = to_gmem((V *)d.cv);
                    for (int i = lane; i < runs; i += 64) {
                        const K k = L.key[i];
                        cri[c0 + out + total + i] = (int32_t)(k >> kKeyBits);
                        cv[c0 + out + total + i] = L.val[(int)(k & (K)(N - 1))];
                    }
                }
                wsync();
            }
            total += runs;
        }
        if (!FILL && lane == 0) {
            a.wcnt[wb + w] = total;
            atomicAdd(&a.gnnz[g], total);
        }
        if (FILL && a.spec_fill && lane == 0) {
            // at a previous structure's positions: the window must have kept
            // its count
            if (total != a.wcnt[wb + w]) bad = 1;
            atomicAdd(&a.gnnz[g], total);
        }
        wsync();
    }
    if (__builtin_amdgcn_ballot_w64(bad != 0) && lane == 0)
        atomicOr(&a.hdr->err, FILL && a.spec_fill ? ERR_RETRY : ERR_GROUP);
}

// ---------------------------------------------------------------- launchers
// ESC sub-bins 0 and 1 (at most 4, 8 products): one column per lane. ESC
// sub-bin i >= 2 (at most 4 << i products): KPL = 4 (256 positions), segments
// of 4 << i (measured: segments of 16 beat a lane per column by 16%, segments
// of 8 lose by 14%). Sort bins 0 and 1 (at most 512, 1024 products): one
// column per wave, KPL = 8, 16. Larger columns are heavy.
template <typename K, typename V, bool FILL>
static hipError_t launch_wave_bin(const KArgs &a, int bin, int grid, hipStream_t s) {
    const dim3 g(grid), t(64);
    switch (bin) {
        case BIN_ESC0 + 0: hipLaunchKernelGGL((k_acc_lane<K, V, 4, FILL>), g, t, 0, s, a, bin); break;
        case BIN_ESC0 + 1: hipLaunchKernelGGL((k_acc_lane<K, V, 8, FILL>), g, t, 0, s, a, bin); break;
        case BIN_ESC0 + 2: hipLaunchKernelGGL((k_acc_wave<K, V, 4, 16, FILL>), g, t, 0, s, a, bin); break;
        case BIN_ESC0 + 3: hipLaunchKernelGGL((k_acc_wave<K, V, 4, 32, FILL>), g, t, 0, s, a, bin); break;
        case BIN_ESC0 + 4: hipLaunchKernelGGL((k_acc_wave<K, V, 4, 64, FILL>), g, t, 0, s, a, bin); break;
        case BIN_ESC0 + 5: hipLaunchKernelGGL((k_acc_wave<K, V, 4, 128, FILL>), g, t, 0, s, a, bin); break;
        case BIN_ESC0 + 6: hipLaunchKernelGGL((k_acc_wave<K, V, 4, 256, FILL>), g, t, 0, s, a, bin); break;
        case BIN_SORT0 + 0: hipLaunchKernelGGL((k_acc_wave<K, V, 8, 512, FILL>), g, t, 0, s, a, bin); break;
        case BIN_SORT0 + 1: hipLaunchKernelGGL((k_acc_wave<K, V, 16, 1024, FILL>), g, t, 0, s, a, bin); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// work items of a wave bin: 64 columns (one per lane: ESC sub-bins 0 and 1),
// groups of columns (the other ESC sub-bins) or columns (sort bins)
int wave_bin_items(int bin, int ncols) {
    if (bin >= BIN_ESC0 && bin < BIN_ESC0 + kLaneSubBins) return ceil_div(ncols, 64);
    if (bin >= BIN_ESC0 && bin < BIN_ESC0 + kEscBins) return ceil_div(ncols, 64 >> (bin - BIN_ESC0));
    return ncols;
}

hipError_t launch_acc_wave(const KArgs &a, int bin, int items, bool wide, bool fill, bool f64,
                           hipStream_t s) {
    if (items <= 0) return hipSuccess;
    if (!fill) {
        return wide ? launch_wave_bin<unsigned long long, float, false>(a, bin, items, s)
                    : launch_wave_bin<unsigned, float, false>(a, bin, items, s);
    }
    if (f64)
        return wide ? launch_wave_bin<unsigned long long, double, true>(a, bin, items, s)
                    : launch_wave_bin<unsigned, double, true>(a, bin, items, s);
    return wide ? launch_wave_bin<unsigned long long, float, true>(a, bin, items, s)
                : launch_wave_bin<unsigned, float, true>(a, bin, items, s);
}

hipError_t launch_heavy_plan(const KArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_heavy_plan, dim3(1), dim3(1024), 0, s, a);
    return hipGetLastError();
}

// The heavy columns' launches one part at a time (the caller interleaves them
// with other streams' launches): windows take the map of windows, the
// expansion and the windowed sort; the radix ESC the expansion and the sort.
int heavy_parts(bool radix) { return radix ? 2 : 3; }
// the first part a launch needs: the windows' map is written by the heavy
// plan of a planned launch
int heavy_first_part(bool radix, bool planned) { return !radix && planned ? 1 : 0; }

hipError_t launch_heavy(const KArgs &a, int ncols, int nwin, bool wide, bool fill, bool f64,
                        hipStream_t s, bool radix, long long heavy_products, int rowbits,
                        int part) {
    if (ncols <= 0) return hipSuccess;
    const bool expand = radix ? part == 0 : part == 1;
    if (expand) {
        if (!fill) hipLaunchKernelGGL((k_heavy_expand<float, false>), dim3(ncols), dim3(kBlock), 0, s, a);
        else if (f64) hipLaunchKernelGGL((k_heavy_expand<double, true>), dim3(ncols), dim3(kBlock), 0, s, a);
        else hipLaunchKernelGGL((k_heavy_expand<float, true>), dim3(ncols), dim3(kBlock), 0, s, a);
        return hipGetLastError();
    }
    if (radix) return part == 1 ? launch_esc_radix(a, heavy_products, rowbits, fill, f64, s) : hipSuccess;
    if (part == 0) {
        hipLaunchKernelGGL(k_win_map, dim3(ceil_div(ncols, kBlock)), dim3(kBlock), 0, s, a);
        return hipGetLastError();
    }
    if (part != 2 || nwin <= 0) return hipSuccess;
    if (!fill) {
        if (wide) hipLaunchKernelGGL((k_acc_window<unsigned long long, float, false>), dim3(nwin), dim3(64), 0, s, a);
        else hipLaunchKernelGGL((k_acc_window<unsigned, float, false>), dim3(nwin), dim3(64), 0, s, a);
    } else if (f64) {
        if (wide) hipLaunchKernelGGL((k_acc_window<unsigned long long, double, true>), dim3(nwin), dim3(64), 0, s, a);
        else hipLaunchKernelGGL((k_acc_window<unsigned, double, true>), dim3(nwin), dim3(64), 0, s, a);
    } else {
        if (wide) hipLaunchKernelGGL((k_acc_window<unsigned long long, float, true>), dim3(nwin), dim3(64), 0, s, a);
        else hipLaunchKernelGGL((k_acc_window<unsigned, float, true>), dim3(nwin), dim3(64), 0, s, a);
    }
    return hipGetLastError();
}

}  // namespace spg
