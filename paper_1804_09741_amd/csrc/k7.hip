// k = 7.  Section 1 counts 880,471,142 classes of 7-vertex digraphs; a code
// -> class table would need 2^42 entries, so here the class of a subgraph is
// its canonical code (the minimum adjacency code over the 5040 relabelings,
// the rule the k <= 6 tables are built by), and H_7 of a graph is a set of
// (canonical code, count) pairs.
//
// The walk is the enumeration kernel's (ESU with per-wave marks, the last
// two levels flat: pairs inside a small extension list per pair of cells,
// other pairs by arc test, exclusive neighbours by list scan), with 42-bit
// codes; as there, graphs past the LDS limit keep their marks in device
// memory and test arcs on the sorted lists (k7_kernel<kVarSearch |
// kVarGlobal>).  Codes go into a
// per-wave LDS hash of pending counts; at its flush each distinct labeled
// code gets its canonical code from a device-wide cache (labeled ->
// canonical, open addressing); a code not in the cache is canonicalised by
// the whole wave -- each lane tries 79 of the 5040 relabelings, then a
// minimum over the wave -- and entered.  Counts are added to the graph's
// class table (canonical code -> u64 count, open addressing).
#include "esu.h"

namespace mk {

using Code7 = unsigned long long;
constexpr Code7 kNoCode = ~0ull;       // free slot / value not written yet
#ifndef MK_K7_HASH_BITS
#define MK_K7_HASH_BITS 8
#endif
constexpr int kHash7Bits = MK_K7_HASH_BITS;    // per-wave LDS hash: 2^bits slots
constexpr int kHash7Slots = 1 << kHash7Bits;
constexpr int kHash7Probes = 8;
constexpr int kCacheProbes = 32;
constexpr int kClassProbes = 64;

struct K7Tables {
    Code7 *cache_key;              // labeled code (kNoCode: free)
    Code7 *cache_val;              // its canonical code (kNoCode: not written yet)
    int cache_shift;               // 64 - log2(cache slots)
    uint32_t cache_mask;
    Code7 *class_key;              // per graph class_mask + 1 canonical codes
    unsigned long long *class_cnt; //   and their counts
    int class_shift;               // 64 - log2(class slots)
    uint32_t class_mask;
    unsigned long long *totals;    // per graph: subgraphs counted
    uint32_t *overflow;            // class-table inserts that found no slot
    uint32_t *cache_used;          // cache slots claimed so far (its fill level)
    uint8_t *etag;                 // marks in device memory: the tags too,
    size_t etag_stride;            //   etag_stride bytes per workgroup, zero
};

// per-wave hash of pending (labeled code, count) pairs in LDS
struct K7Wave {
    Code7 *hkey;
    uint32_t *hcnt;    // 32-bit two's complement counts (corrections are negative)
    int hused;
    uint32_t hpending;
    int graph;
    uint8_t *etag;     // per vertex: 0x80 | lane while it is in a small node's E
                       // (LDS, or device memory with the marks)
    Code7 *cc1, *cc2;  // per cell of E: code bits at positions 5 and 6
    uint32_t *csz;     //   and its size
};

__device__ __forceinline__ uint32_t hash7(Code7 c, int shift)
{
    return (uint32_t)((c * 0x9E3779B97F4A7C15ull) >> shift);
}

__device__ __forceinline__ Code7 readlane64(Code7 v, int l)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
    return ((Code7)hi << 32) | lo;
}

// position of arc i -> j in a 7-vertex code
__host__ __device__ constexpr int bit7(int i, int j) { return i * 6 + j - (j > i ? 1 : 0); }

// code bits of a vertex with mark m joining at position p (1..6)
__device__ __forceinline__ Code7 code_bits7(uint32_t m, int p)
{
    return ((Code7)(m >> EnumState<7>::OUTB) << (p * 6)) |
           ((Code7)(m & EnumState<7>::INMASK) << (p - 1));
}

// i-th set bit (0-based) of a 7-bit mask
__device__ __forceinline__ uint32_t nth_bit(uint32_t m, int i)
{
    for (int t = 0; t < i; ++t) m &= m - 1u;
    return (uint32_t)__builtin_ctz(m);
}

// out-neighbours of vertex c in a 7-vertex code (row c, column r is vertex
// r + [r >= c]), as a 7-bit mask
__device__ __forceinline__ uint32_t out_nbrs7(Code7 code, uint32_t c)
{
    const uint32_t row = (uint32_t)((code >> (6 * c)) & 63ull);
    const uint32_t lowc = (1u << c) - 1u;
    return (row & lowc) | ((row & ~lowc) << 1);
}

// the vertices of mask m in increasing order take positions first.. in the
// order numbered r (factorial number system), into the 4-bit fields of sigma
__device__ __forceinline__ void place7(uint32_t &sigma, uint32_t m, int first, int count, int r)
{
    constexpr int fact[7] = {1, 1, 2, 6, 24, 120, 720};
    for (int pos = 0; pos < count; ++pos) {
        const int f = fact[count - 1 - pos];
        const int d = r / f;
        r -= d * f;
        const uint32_t v = nth_bit(m, d);
        sigma |= (uint32_t)(first + pos) << (4 * v);
        m &= ~(1u << v);
    }
}

// Canonical code: the minimum code over the relabelings.  Only relabelings
// that can reach the minimum are tried.  The top six bits of a code are the
// out-arcs of the vertex at position 6 (bit of arc 6 -> j at 36 + j); for a
// vertex of out-degree d they are at least 2^d - 1, reached exactly when its
// out-neighbours take positions 0..d-1.  So the minimum puts at position 6
// a vertex of the least out-degree d6 and its out-neighbours at 0..d6-1.
// When d6 = 0 (a sink at 6, the usual case in sparse graphs) the next six
// bits are the row of position 5, whose top bit is its arc to position 6:
// the minimum puts at 5 a vertex without that arc if there is one, of the
// least out-degree d5 towards the other five among those, and its
// out-neighbours at 0..d5-1.  For each candidate at position 6 in turn, the
// relabelings left are numbered (the candidate at 5, then the order of each
// group of positions in the factorial number system); lane l tries l,
// l + 64, ..., and the wave takes the minimum.  Call with every lane active
// and the same code in all lanes.
__device__ __forceinline__ Code7 canon7_wave(Code7 code)
{
    constexpr int fact[7] = {1, 1, 2, 6, 24, 120, 720};
    uint32_t c6m = 0;
    int d6 = 7;
#pragma unroll
    for (int i = 0; i < 7; ++i) {
        const int od = __builtin_popcountll((code >> (6 * i)) & 63ull);
        if (od < d6) {
            d6 = od;
            c6m = 0;
        }
        if (od == d6) c6m |= 1u << i;
    }
    Code7 best = kNoCode;
    // one candidate for position 6 at a time (wave-uniform)
    for (uint32_t left6 = c6m; left6; left6 &= left6 - 1u) {
        const uint32_t c6 = (uint32_t)__builtin_ctz(left6);
        // d6 = 0: the candidates for position 5 and their out-degree d5
        uint32_t c5m = 0;
        int d5 = 0, cnt = fact[d6] * fact[6 - d6];
        if (d6 == 0) {
            int key_min = 64;
            for (uint32_t v = 0; v < 7; ++v) {
                if (v == c6) continue;
                const uint32_t on = out_nbrs7(code, v);
                const int key = (int)(((on >> c6) & 1u) << 3) + __builtin_popcount(on & ~(1u << c6));
                if (key < key_min) {
                    key_min = key;
                    c5m = 0;
                }
                if (key == key_min) c5m |= 1u << v;
            }
            d5 = key_min & 7;
            cnt = __builtin_popcount(c5m) * fact[d5] * fact[5 - d5];
        }
        for (int t = lane_id(); t < cnt; t += kWave) {
            uint32_t sigma = 6u << (4 * c6);
            int r = t;
            if (d6 > 0) {
                const uint32_t on = out_nbrs7(code, c6);
                const int q = r / fact[6 - d6];
                place7(sigma, on, 0, d6, q);
                place7(sigma, 0x7Fu & ~on & ~(1u << c6), d6, 6 - d6, r - q * fact[6 - d6]);
            } else {
                const int per = fact[d5] * fact[5 - d5];
                const uint32_t c5 = nth_bit(c5m, r / per);
                r %= per;
                sigma |= 5u << (4 * c5);
                const uint32_t on = out_nbrs7(code, c5) & ~(1u << c6);
                const int q = r / fact[5 - d5];
                place7(sigma, on, 0, d5, q);
                place7(sigma, 0x7Fu & ~on & ~(1u << c6) & ~(1u << c5), d5, 5 - d5,
                       r - q * fact[5 - d5]);
            }
            Code7 cc = 0, rest = code;
            while (rest) {
                const int b = __builtin_ctzll(rest);
                rest &= rest - 1;
                const int i = b / 6, rr = b - 6 * i;
                const int j = rr + (rr >= i ? 1 : 0);
                cc |= 1ull << bit7((int)((sigma >> (4 * i)) & 15u), (int)((sigma >> (4 * j)) & 15u));
            }
            best = cc < best ? cc : best;
        }
    }
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        const Code7 o = __shfl_xor(best, off, kWave);
        best = o < best ? o : best;
    }
    return best;
}

// Move the wave's pending counts to its graph's class table: canonical code
// from the cache (or computed and entered), count added; hash emptied.
template <int V>
__device__ __forceinline__ void flush7(EnumState<7, V> &s, K7Wave &w, const K7Tables &t)
{
    __syncthreads();
    const int lane = lane_id();
    unsigned long long tot = 0;
    Code7 *ckey = t.class_key + (size_t)w.graph * (t.class_mask + 1);
    unsigned long long *ccnt = t.class_cnt + (size_t)w.graph * (t.class_mask + 1);
    for (int base = 0; base < kHash7Slots; base += kWave) {
        const int i = base + lane;
        const Code7 key = w.hkey[i];
        const uint32_t cnt = w.hcnt[i];
        const bool live = key != kNoCode;
        Code7 canon = kNoCode;
        if (live) {
            uint32_t h = hash7(key, t.cache_shift);
            for (int p = 0; p < kCacheProbes; ++p) {
                const Code7 k2 = t.cache_key[h];
                if (k2 == key) {
                    canon = t.cache_val[h];
                    break;
                }
                if (k2 == kNoCode) break;
                h = (h + 1) & t.cache_mask;
            }
        }
        const bool missed = live && canon == kNoCode;
        unsigned long long miss = __ballot(missed);
        while (miss) {
            const int l = __builtin_ctzll(miss);
            miss &= miss - 1;
            const Code7 m = canon7_wave(readlane64(key, l));
            if (lane == l) canon = m;
        }
        bool claimed = false;
        if (missed) {
            // enter it: the lane that claims the key writes the value; a
            // reader that meets the key before the value computes it again
            uint32_t h = hash7(key, t.cache_shift);
            for (int p = 0; p < kCacheProbes; ++p) {
                const Code7 old = atomicCAS(&t.cache_key[h], kNoCode, key);
                if (old == kNoCode) {
                    atomicExch(&t.cache_val[h], canon);
                    claimed = true;
                    break;
                }
                if (old == key) break;
                h = (h + 1) & t.cache_mask;
            }
        }
        const unsigned long long ins = __ballot(claimed);
        if (lane == 0 && ins) atomicAdd(t.cache_used, (uint32_t)__popcll(ins));
        if (live && cnt != 0u) {
            // sign-extended: the 64-bit sums stay exact modulo 2^64
            const unsigned long long add = (unsigned long long)(long long)(int32_t)cnt;
            uint32_t h = hash7(canon, t.class_shift);
            bool done = false;
            for (int p = 0; p < kClassProbes && !done; ++p) {
                const Code7 old = atomicCAS(&ckey[h], kNoCode, canon);
                if (old == kNoCode || old == canon) {
                    atomicAdd(&ccnt[h], add);
                    done = true;
                }
                h = (h + 1) & t.class_mask;
            }
            if (!done) atomicAdd(t.overflow, 1u);
            tot += add;
        }
        if (live) {
            w.hkey[i] = kNoCode;
            w.hcnt[i] = 0u;
        }
    }
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) tot += __shfl_xor(tot, off, kWave);
    if (lane == 0 && tot) atomicAdd(&t.totals[w.graph], tot);
    w.hused = 0;
    w.hpending = 0;
    __syncthreads();
}

// add n to the pending count of code for every lane with `mine` set; a full
// hash is flushed and the inserts that found no slot are tried again
template <int V>
__device__ __forceinline__ void hash7_insert(EnumState<7, V> &s, K7Wave &w, const K7Tables &t, bool mine, Code7 code,
                             uint32_t n)
{
    bool pending = mine;
    for (;;) {
        bool fresh = false;
        if (pending) {
            uint32_t h = hash7(code, 64 - kHash7Bits);
            for (int p = 0; p < kHash7Probes; ++p) {
                const Code7 old = atomicCAS(&w.hkey[h], kNoCode, code);
                if (old == kNoCode || old == code) {
                    fresh = old == kNoCode;
                    atomicAdd(&w.hcnt[h], n);
                    pending = false;
                    break;
                }
                h = (h + 1) & (kHash7Slots - 1);
            }
        }
        w.hused += __popcll(__ballot(fresh));
        const bool retry = __ballot(pending) != 0ull;
        if (retry || w.hused > kHash7Slots / 2 || w.hpending >= kPendingMax) flush7(s, w, t);
        if (!retry) break;
    }
}

// count one code per valid lane (lanes sharing the first lane's code merged)
template <int V>
__device__ __forceinline__ void count7(EnumState<7, V> &s, K7Wave &w, const K7Tables &t, bool valid, Code7 code)
{
    const int lane = lane_id();
    const unsigned long long act = __ballot(valid);
    if (!act) return;
    w.hpending += (uint32_t)__popcll(act);
    const int l = __builtin_ctzll(act);
    const Code7 c0 = readlane64(code, l);
    const unsigned long long eq = __ballot(valid && code == c0) & act;
    uint32_t n = 1;
    if (lane == l) n = (uint32_t)__popcll(eq);
    else if ((eq >> lane) & 1ull) n = 0;
    hash7_insert(s, w, t, valid && n > 0, code, n);
}

// count each valid lane's code with weight -1 (merged like count7)
template <int V>
__device__ __forceinline__ void uncount7(EnumState<7, V> &s, K7Wave &w, const K7Tables &t, bool valid, Code7 code)
{
    const int lane = lane_id();
    const unsigned long long act = __ballot(valid);
    if (!act) return;
    w.hpending += (uint32_t)__popcll(act);
    const int l = __builtin_ctzll(act);
    const Code7 c0 = readlane64(code, l);
    const unsigned long long eq = __ballot(valid && code == c0) & act;
    uint32_t n = 1;
    if (lane == l) n = (uint32_t)__popcll(eq);
    else if ((eq >> lane) & 1ull) n = 0;
    hash7_insert(s, w, t, valid && n > 0, code, 0u - n);
}

// position in seg storage of element a of the extension list made of the
// tails seg[q][st[q]:], q < NQ
template <int NQ, int V>
__device__ __forceinline__ int ext_addr7(const EnumState<7, V> &s, const int (&st)[6],
                                         const int (&rem)[NQ], int a)
{
    int addr = 0;
    bool found = false;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        if (!found) {
            if (a < rem[q]) {
                addr = q * s.seg_cap + st[q] + a;
                found = true;
            } else {
                a -= rem[q];
            }
        }
    }
    return addr;
}

// lane l's value of v (every lane active: a permute reads 0 from an
// inactive lane)
__device__ __forceinline__ uint32_t from_lane7(uint32_t v, int l)
{
    return (uint32_t)__builtin_amdgcn_ds_bpermute(l << 2, (int)v);
}

__device__ __forceinline__ Code7 from_lane64(Code7 v, int l)
{
    return ((Code7)from_lane7((uint32_t)(v >> 32), l) << 32) | from_lane7((uint32_t)v, l);
}

// Nodes with at most one wave of extension vertices: the pairs inside E are
// counted per pair of cells, as in Section 3's loop over L_{k-2}.  Vertices
// of E with equal marks relate alike to the members, so all pairs from
// cells A and B without an arc between them have one class; there are
// C(n_A, 2) or n_A n_B of them.  The arcs inside E are found while the
// children's lists are scanned for their exclusive neighbours: E's vertices
// carry a tag with their lane meanwhile, and each arc (w, u), u after w,
// adds one to its own code and takes one from its cell pair's.  Lane l holds
// E[l], its code bits for positions 5 and 6 and its list row; a child of
// degree >= kRowMin is scanned alone.
template <int V>
__device__ __forceinline__ void last_two7_cells(EnumState<7, V> &s, K7Wave &w7, const K7Tables &t, const int (&st)[6],
                                const int (&rem)[5], int e, Code7 code, int jlo)
{
    constexpr int B_WU = bit7(5, 6), B_UW = bit7(6, 5);
    const int lane = lane_id();
    const bool inE = lane >= jlo && lane < e;
    uint32_t vtx = 0;
    Code7 cb1 = 0, cb2 = 0;
    int row = 0, deg = 0;
    if (lane < e) {
        vtx = s.seg[ext_addr7<5>(s, st, rem, lane)];
        const uint32_t m = s.mark[vtx];
        cb1 = code_bits7(m, 5);
        cb2 = code_bits7(m, 6);
        row = s.urow[vtx];
        deg = s.urow[vtx + 1] - row;
    }
    if (!inE) deg = 0;
    if (inE) w7.etag[vtx] = (uint8_t)(0x80u | (uint32_t)lane);
    __syncthreads();
    auto tbits = [](uint32_t tt) { return ((Code7)(tt & 1u) << B_WU) | ((Code7)(tt >> 1) << B_UW); };

    // children with long lists alone: exclusive neighbours by arc type, arcs
    // to later vertices of E one by one
    unsigned long long big = __ballot(deg >= kRowMin);
    while (big) {
        const int l = __builtin_ctzll(big);
        big &= big - 1;
        const int brow = __builtin_amdgcn_readlane(row, l);
        const int bdeg = __builtin_amdgcn_readlane(deg, l);
        const Code7 bcode = code | readlane64(cb1, l);
        uint32_t n1 = 0, n2 = 0, n3 = 0;
        for (int b = 0; b < bdeg; b += kWave) {
            const int e2 = b + lane;
            uint32_t tb = 0, tt = 0;
            bool arc = false;
            int q = 0;
            if (e2 < bdeg) {
                const uint32_t ent = s.uadj[brow + e2];
                const int u = (int)(ent >> 2);
                const uint32_t tg = w7.etag[u];
                tt = ent & 3u;
                if (tg & 0x80u) {
                    q = (int)(tg & 63u);
                    arc = q > l;
                } else if (u > s.root && s.mark[u] == 0u) {
                    tb = tt;
                }
            }
            n1 += (uint32_t)__popcll(__ballot(tb == 1u));
            n2 += (uint32_t)__popcll(__ballot(tb == 2u));
            n3 += (uint32_t)__popcll(__ballot(tb == 3u));
            const Code7 cm = bcode | from_lane64(cb2, q);
            count7(s, w7, t, arc, cm | tbits(tt));
            uncount7(s, w7, t, arc, cm);
        }
        const uint32_t tl = (uint32_t)lane + 1u;
        const uint32_t nl = lane == 0 ? n1 : (lane == 1 ? n2 : n3);
        w7.hpending += n1 + n2 + n3;
        hash7_insert(s, w7, t, lane < 3 && nl > 0, bcode | tbits(tl), nl);
    }
    if (deg >= kRowMin) deg = 0;
    int incl = deg;
    incl = wave_incl_sum(incl);
    const int totB = __builtin_amdgcn_readlane(incl, kWave - 1);
    uint32_t *pre = s.scratch;  // flat_source's buffer
    // flat entry f of this lane's list sits at rowb + f
    const int rowb = row - (incl - deg);
    // the short lists, flat: exclusive neighbours and arcs inside E
    for (int base = 0; base < totB; base += kWave) {
        const int f = base + lane;
        const bool valid = f < totB;
        const int src1 = flat_source(pre, incl, deg, base);
        const int off = f;
        // the permutes run with every lane active
        const int r1 = (int)from_lane7((uint32_t)rowb, src1);
        const Code7 c1 = from_lane64(cb1, src1);
        bool bv = false, arc = false;
        uint32_t tt = 0;
        int q = 0;
        if (valid) {
            const uint32_t ent = s.uadj[r1 + off];
            const int u = (int)(ent >> 2);
            const uint32_t tg = w7.etag[u];
            tt = ent & 3u;
            if (tg & 0x80u) {
                q = (int)(tg & 63u);
                arc = q > src1;
            } else {
                bv = u > s.root && s.mark[u] == 0u;
            }
        }
        const Code7 cm = code | c1 | from_lane64(cb2, q);
        count7(s, w7, t, bv, code | c1 | tbits(tt));
        count7(s, w7, t, arc, cm | tbits(tt));
        uncount7(s, w7, t, arc, cm);
    }
    __syncthreads();

    // the cells of E (vertices with equal marks) and their pairs
    const Code7 key = inE ? cb1 : kNoCode;
    unsigned long long left = __ballot(inE);
    bool leader = false;
    uint32_t size = 0;
    while (left) {
        const int l = __builtin_ctzll(left);
        const Code7 k0 = readlane64(key, l);
        const unsigned long long eq = __ballot(key == k0) & left;
        if (lane == l) {
            leader = true;
            size = (uint32_t)__popcll(eq);
        }
        left &= ~eq;
    }
    const unsigned long long leaders = __ballot(leader);
    const int ncell = __popcll(leaders);
    if (leader) {
        const int rk = (int)lanes_below(leaders);
        w7.cc1[rk] = cb1;
        w7.cc2[rk] = cb2;
        w7.csz[rk] = size;
    }
    __syncthreads();
    const int mm = e - jlo;
    const uint32_t all_pairs = (uint32_t)(mm * (mm - 1) / 2);
    if (w7.hpending + all_pairs >= kPendingMax) flush7(s, w7, t);
    w7.hpending += all_pairs;
    const int ncp = ncell * (ncell + 1) / 2;
    for (int pb = 0; pb < ncp; pb += kWave) {
        const int p = pb + lane;
        bool valid = p < ncp;
        Code7 c = 0;
        uint32_t w = 0;
        if (valid) {
            // p = z(z+1)/2 + y with y <= z
            int z = (int)((__builtin_amdgcn_sqrtf(8.0f * (float)p + 1.0f) - 1.0f) * 0.5f);
            if ((z + 1) * (z + 2) / 2 <= p) ++z;
            if (z * (z + 1) / 2 > p) --z;
            const int y = p - z * (z + 1) / 2;
            const uint32_t ny = w7.csz[y], nz = w7.csz[z];
            w = y == z ? ny * (ny - 1u) / 2u : ny * nz;
            c = code | w7.cc1[y] | w7.cc2[z];
            valid = w > 0u;
        }
        hash7_insert(s, w7, t, valid, c, w);
    }
    if (inE) w7.etag[vtx] = 0;
    __syncthreads();
}

// The last two levels of a node X with members s_0..s_4 and extension list
// E: child w = E[i] (i in [jlo, jhi)) closes X + {w, u} for (A) u = E[j],
// j > i (arc w - u from the bit matrices) and (B) u an exclusive neighbour
// of w (its list entry gives the arc).  Same split as the k <= 6 kernel.
template <int V>
__device__ __forceinline__ void last_two7(EnumState<7, V> &s, K7Wave &w7, const K7Tables &t, const int (&st)[6],
                          Code7 code, int jlo, int jhi)
{
    constexpr int NQ = 5;
    constexpr int B_WU = bit7(5, 6);  // arc s_5 -> s_6
    constexpr int B_UW = bit7(6, 5);  // arc s_6 -> s_5
    const int lane = lane_id();
    int rem[NQ];
    int e = 0;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        rem[q] = s.len[q] - st[q];
        e += rem[q];
    }
    const int hi = e < jhi ? e : jhi;
    if (jlo >= hi) return;
    if (e <= kWave && hi == e) {
        last_two7_cells(s, w7, t, st, rem, e, code, jlo);
        return;
    }

    // (A) pairs (E[i], E[j]), jlo <= i < hi, i < j < e, row by row
    const int rows = hi - jlo;
    const int A = e - 1 - jlo;
    const long long npairs = (long long)rows * A - (long long)rows * (rows - 1) / 2;
    const float tA = 2.0f * (float)A + 1.0f;
    for (long long base = 0; base < npairs; base += kWave) {
        const long long p = base + lane;
        const bool valid = p < npairs;
        Code7 c = 0;
        bool ok = false;
        if (valid) {
            float disc = tA * tA - 8.0f * (float)p;
            disc = disc > 0.f ? disc : 0.f;
            int r = (int)((tA - __builtin_amdgcn_sqrtf(disc)) * 0.5f);
            r = r < 0 ? 0 : (r > rows - 1 ? rows - 1 : r);
            while (r + 1 < rows && (long long)(r + 1) * A - (long long)(r + 1) * r / 2 <= p) ++r;
            while (r > 0 && (long long)r * A - (long long)r * (r - 1) / 2 > p) --r;
            const int i = jlo + r;
            const int j = i + 1 + (int)(p - ((long long)r * A - (long long)r * (r - 1) / 2));
            if (i < j && j < e) {
                const uint32_t w = s.seg[ext_addr7<NQ>(s, st, rem, i)];
                const uint32_t u = s.seg[ext_addr7<NQ>(s, st, rem, j)];
                uint32_t tt;
                if constexpr ((V & kVarSearch) != 0) {
                    tt = list_relation(s.urow, s.uadj, w, u);
                } else {
                    const size_t word = (size_t)w * s.words + (u >> 5);
                    const uint32_t sh = u & 31u;
                    tt = ((s.bits_out[word] >> sh) & 1u) | (((s.bits_in[word] >> sh) & 1u) << 1);
                }
                c = code | code_bits7(s.mark[w], 5) | code_bits7(s.mark[u], 6) |
                    ((Code7)(tt & 1u) << B_WU) | ((Code7)(tt >> 1) << B_UW);
                ok = true;
            } else {
                atomicAdd(s.errors, 1u);  // unreachable: the decode keeps i < j < e
            }
        }
        count7(s, w7, t, ok, c);
    }

    // (B) exclusive neighbours, 64 children at a time: a lane-prefix sum of
    // their degrees maps a flat index to (child, list position)
    uint32_t *pre = s.scratch, *start = s.scratch + kWave;
    for (int ib = jlo; ib < hi; ib += kWave) {
        const int i = ib + lane;
        int deg = 0, row = 0;
        Code7 wcode = 0;
        if (i < hi) {
            const uint32_t w = s.seg[ext_addr7<NQ>(s, st, rem, i)];
            row = s.urow[w];
            deg = s.urow[w + 1] - row;
            wcode = code_bits7(s.mark[w], 5);
        }
        int incl = deg;
        incl = wave_incl_sum(incl);
        const int tot = __builtin_amdgcn_readlane(incl, kWave - 1);
        start[lane] = (uint32_t)(row - (incl - deg));  // flat entry f at start + f
        __syncthreads();
        for (int fb = 0; fb < tot; fb += kWave) {
            const int f = fb + lane;
            bool valid = f < tot;
            const int lo = flat_source(pre, incl, deg, fb);
            // the child's code bits from its lane (every lane active here)
            const Code7 cw = ((Code7)(uint32_t)__builtin_amdgcn_ds_bpermute(
                                  lo << 2, (int)(uint32_t)(wcode >> 32)) << 32) |
                             (uint32_t)__builtin_amdgcn_ds_bpermute(lo << 2, (int)(uint32_t)wcode);
            Code7 c = 0;
            if (valid) {
                const uint32_t ent = s.uadj[start[lo] + (uint32_t)f];
                const int u = (int)(ent >> 2);
                const uint32_t tt = ent & 3u;
                valid = u > s.root && s.mark[u] == 0u;
                c = code | cw | ((Code7)(tt & 1u) << B_WU) | ((Code7)(tt >> 1) << B_UW);
            }
            count7(s, w7, t, valid, c);
        }
        __syncthreads();
    }
}

// node with members s_0..s_D: children jlo..jhi-1 of its extension list
template <int D, int V>
__device__ __forceinline__ void visit7(EnumState<7, V> &s, K7Wave &w7, const K7Tables &t, const int (&st)[6],
                       Code7 code, int jlo, int jhi)
{
    if constexpr (D == 4) {
        last_two7(s, w7, t, st, code, jlo, jhi);
    } else {
        int rem[D + 1];
        int total = 0;
#pragma unroll
        for (int q = 0; q <= D; ++q) {
            rem[q] = s.len[q] - st[q];
            total += rem[q];
        }
        const int hi = total < jhi ? total : jhi;
        for (int j = jlo; j < hi; ++j) {
            int a = j, L = 0, o = 0;
            bool found = false;
#pragma unroll
            for (int q = 0; q <= D; ++q) {
                if (!found) {
                    if (a < rem[q]) {
                        L = q;
                        o = st[q] + a;
                        found = true;
                    } else {
                        a -= rem[q];
                    }
                }
            }
            const int x = uniform((int)s.seg[L * s.seg_cap + o]);
            const uint32_t mx = (uint32_t)uniform((int)s.mark[x]);
            const Code7 ccode = code | code_bits7(mx, D + 1);
            const Held held = push_held<7, D + 1>(s, x);
            int cst[6];
#pragma unroll
            for (int q = 0; q < 6; ++q)
                cst[q] = q < L ? s.len[q] : (q == L ? o + 1 : (q <= D ? st[q] : 0));
            visit7<D + 1>(s, w7, t, cst, ccode, 0, INT_MAX);
            pop_held<7, D + 1>(s, x, held);
        }
    }
}

template <int V>
__device__ __forceinline__ void run_unit7(EnumState<7, V> &s, K7Wave &w7, const K7Tables &t, int v, int i,
                          uint32_t range)
{
    s.root = v;
    const Held held0 = push_held<7, 0>(s, v);
    if (i < s.len[0]) {
        const int x = uniform((int)s.seg[i]);
        const Code7 code = code_bits7((uint32_t)uniform((int)s.mark[x]), 1);
        const Held held1 = push_held<7, 1>(s, x);
        int st[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) st[q] = 0;
        st[0] = i + 1;
        const bool full = range == kFullChild;
        visit7<1>(s, w7, t, st, code, full ? 0 : (int)(range & 0xFFFFu),
                  full ? INT_MAX : (int)(range >> 16));
        pop_held<7, 1>(s, x, held1);
    } else if (lane_id() == 0) {
        atomicAdd(s.errors, 1u);
    }
    pop_held<7, 0>(s, v, held0);
}

// this kernel's part of a wave's LDS, after the shared layout: the hash
// (u64 keys, u32 counts), the cell table (2 x u64 + u32 per cell), the
// extension tags (a byte per vertex)
static __host__ __device__ int k7_hash_offset(int max_n, int seg_cap, bool global)
{
    return (lds_layout(7, max_n, seg_cap, 0, global).total + 7) & ~7;
}

static __host__ __device__ int k7_cells_offset(int max_n, int seg_cap, bool global)
{
    return k7_hash_offset(max_n, seg_cap, global) +
           kHash7Slots * (int)(sizeof(Code7) + sizeof(uint32_t));
}

static __host__ __device__ int k7_tags_offset(int max_n, int seg_cap, bool global)
{
    return k7_cells_offset(max_n, seg_cap, global) +
           kWave * (int)(2 * sizeof(Code7) + sizeof(uint32_t));
}

// V = 0: LDS marks and tags, bit-matrix arc tests; V = kVarSearch |
// kVarGlobal: marks and tags in device memory, arc tests on the lists
template <int V>
__global__ __launch_bounds__(kWave) void k7_kernel(const DevGraph *graphs, const int4 *units,
                                                   uint32_t unit_cap, uint32_t unit_end,
                                                   uint32_t *counters, K7Tables t, EnumConfig cfg)
{
    constexpr bool kGlobal = (V & kVarGlobal) != 0;
    extern __shared__ uint32_t lds[];
    char *base = reinterpret_cast<char *>(lds);
    EnumState<7, V> s;
    const LdsLayout lay = lds_layout(7, cfg.max_n, cfg.seg_cap, 0, kGlobal);
    init_state(s, base, lay, cfg, counters, nullptr, 0u);
    K7Wave w7;
    w7.hkey = reinterpret_cast<Code7 *>(base + k7_hash_offset(cfg.max_n, cfg.seg_cap, kGlobal));
    w7.hcnt = reinterpret_cast<uint32_t *>(w7.hkey + kHash7Slots);
    w7.cc1 = reinterpret_cast<Code7 *>(base + k7_cells_offset(cfg.max_n, cfg.seg_cap, kGlobal));
    w7.cc2 = w7.cc1 + kWave;
    w7.csz = reinterpret_cast<uint32_t *>(w7.cc2 + kWave);
    if constexpr (kGlobal) {
        // zeroed when allocated; every small node clears the tags it set
        w7.etag = t.etag + (size_t)blockIdx.x * t.etag_stride;
    } else {
        w7.etag = reinterpret_cast<uint8_t *>(base + k7_tags_offset(cfg.max_n, cfg.seg_cap, false));
        for (int i = lane_id(); i < cfg.max_n; i += kWave) w7.etag[i] = 0;
    }
    w7.hused = 0;
    w7.hpending = 0;
    w7.graph = 0;
    for (int i = lane_id(); i < kHash7Slots; i += kWave) {
        w7.hkey[i] = kNoCode;
        w7.hcnt[i] = 0u;
    }
    __syncthreads();

    unit_loop<false>(
        s, graphs, units, unit_cap, unit_end, counters, cfg,
        [&](int v, int i, uint32_t range) { run_unit7(s, w7, t, v, i, range); },
        [&](int gi) {
            if (w7.hused) flush7(s, w7, t);
            w7.graph = gi;
        },
        [] {});
    if (w7.hused) flush7(s, w7, t);
}

// every used class slot with a non-zero count of every graph to (code,
// count) lists; n_out[g] counts them (entries past cap are counted, not
// written)
__global__ void k7_collect_kernel(const Code7 *class_key, const unsigned long long *class_cnt,
                                  uint32_t slots, int64_t cap, Code7 *out_codes,
                                  unsigned long long *out_counts, unsigned long long *n_out)
{
    const int gi = blockIdx.y;
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= slots) return;
    const size_t at = (size_t)gi * slots + i;
    const Code7 key = class_key[at];
    // a class whose corrections cancel keeps a slot with count 0
    if (key == kNoCode || class_cnt[at] == 0ull) return;
    const unsigned long long pos = atomicAdd(&n_out[gi], 1ull);
    if ((long long)pos < cap) {
        out_codes[(size_t)gi * cap + pos] = key;
        out_counts[(size_t)gi * cap + pos] = class_cnt[at];
    }
}

int k7_lds_bytes(int max_n, int seg_cap, int variant)
{
    const bool global = (variant & kVarGlobal) != 0;
    return k7_tags_offset(max_n, seg_cap, global) + (global ? 0 : ((max_n + 3) & ~3));
}

static const void *k7_fn(int variant)
{
    switch (variant) {
    case 0: return reinterpret_cast<const void *>(&k7_kernel<0>);
    case kVarSearch | kVarGlobal:
        return reinterpret_cast<const void *>(&k7_kernel<kVarSearch | kVarGlobal>);
    default: return nullptr;
    }
}

int k7_max_blocks_per_cu(int variant, int lds_bytes, int *blocks)
{
    const void *fn = k7_fn(variant);
    if (!fn) return fail(MK_ERANGE, "no k = 7 kernel for variant %d", variant);
    MK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, fn, kWave, (size_t)lds_bytes));
    return MK_OK;
}

int launch_k7(const DevGraph *d_graphs, const int4 *units, uint32_t unit_cap, uint32_t *counters,
              const K7Launch &a, const EnumConfig &cfg, int grid, int lds_bytes, hipStream_t stream)
{
    if (grid <= 0) return MK_OK;
    K7Tables t;
    t.cache_key = a.cache_key;
    t.cache_val = a.cache_val;
    t.cache_shift = 64 - a.cache_log2;
    t.cache_mask = (1u << a.cache_log2) - 1u;
    t.class_key = a.class_key;
    t.class_cnt = a.class_cnt;
    t.class_shift = 64 - a.class_log2;
    t.class_mask = (1u << a.class_log2) - 1u;
    t.totals = a.totals;
    t.overflow = a.overflow;
    t.cache_used = a.cache_used;
    t.etag = a.etag;
    t.etag_stride = a.etag_stride;
    const void *fn = k7_fn(cfg.variant);
    if (!fn) return fail(MK_ERANGE, "no k = 7 kernel for variant %d", cfg.variant);
    if ((cfg.variant & kVarGlobal) != 0 && (!cfg.marks || !a.etag))
        return fail(MK_EINVAL, "launch_k7: device-memory variant without marks or tags");
    const uint32_t end = kAllUnits;
    EnumConfig c = cfg;
    void *args[] = {(void *)&d_graphs, (void *)&units, (void *)&unit_cap, (void *)&end,
                    (void *)&counters, (void *)&t, (void *)&c};
    MK_HIP(hipLaunchKernel(fn, dim3(grid), dim3(kWave), args, (size_t)lds_bytes, stream));
    return MK_OK;
}

int launch_k7_collect(const K7Launch &a, int ng, int64_t cap, unsigned long long *out_codes,
                      unsigned long long *out_counts, unsigned long long *n_out, hipStream_t stream)
{
    if (ng <= 0) return MK_OK;
    const uint32_t slots = 1u << a.class_log2;
    const dim3 grid((slots + 255) / 256, (unsigned)ng);
    hipLaunchKernelGGL(k7_collect_kernel, grid, dim3(256), 0, stream, a.class_key, a.class_cnt,
                       slots, cap, out_codes, out_counts, n_out);
    MK_HIP(hipGetLastError());
    return MK_OK;
}

}  // namespace mk
