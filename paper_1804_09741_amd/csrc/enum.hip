// Enumeration of connected induced k-subgraphs, their adjacency codes, the
// O(1) class lookup (Section 3.2) and the histogram H_k (Problem Motifs-k).
//
// One 64-lane wavefront is one workgroup.  Waves are persistent: each takes
// work units from global queues until they are empty.  The unit list is cut
// into eight ranges with a head each (one per XCD, on separate cache lines);
// a wave starts on the range of its own XCD (workgroups are dealt to the
// XCDs round-robin, so consecutive units of one graph stay in one L2) and
// then helps the others.  Units are grabbed a few at a time, so the head
// atomics stay far below their throughput limit.
// A unit is a first-level ESU node (root v, first extension vertex w_i),
// possibly restricted to a range of that node's children (hub splitting).
//
// Per wave, LDS holds
//   mark[n]        for every vertex x, its relation to the current members
//                  s_0..s_d of the growing subgraph: "in" bit d(k-1) set iff
//                  arc s_d -> x, "out" bit OUTB+d set iff arc x -> s_d.  The
//                  in bits are already spread at stride k-1, so the code
//                  bits that a vertex adds when it joins at position p are
//                      (out << p(k-1)) | (in << (p-1))
//                  -- exactly bits b(i,p) = i(k-1)+p-1 and b(p,i) = p(k-1)+i
//                  of the adjacency code.  mark[x] == 0 also says "x is
//                  neither a member nor a neighbour of one" (the exclusive
//                  neighbourhood test of ESU).
//   seg[l][.]      the vertices that joined the extension list when member
//                  s_l was added (s_0's are the root's larger neighbours).
// A node's extension list is the concatenation of the unconsumed tails of
// seg[0..d]; it is never copied.
//
// Adding a member scans its typed adjacency list (Section 2's A/B/C types)
// with all 64 lanes: each lane reads the mark of one neighbour, a ballot and
// a lane-prefix count compact the new extension vertices into seg[d], and the
// lane ORs the member's two bits into the neighbour's mark.  Removing it
// clears those bits again, so marks are all zero between units.
//
// At the last level every extension vertex u closes one k-subgraph: lanes
// take one u each, read mark[u] and form the code with two shifts and an OR
// -- this replaces the pair tests of Algorithms 2-5 (Section 3.1): the edges
// of G[S] are known from the marks the members left.  Codes go into a small
// per-wave LDS hash of pending counts (one ballot round first merges the
// lanes that share the first lane's code): the same few shapes recur across
// nodes, so the hash absorbs most of them, and only its flush looks codes up
// in the code -> class table and adds to the graph's histogram with 64-bit
// atomics.
//
// Two variants of the walk are separate kernels (enum_lists_kernel<k, V>):
// arcs between two extension vertices tested by a binary search in the
// shorter sorted list instead of a bit-matrix read, and, for graphs whose
// marks do not fit LDS, each wave's marks kept in its own array in device
// memory (the kVar* bits).
#include "esu.h"

namespace mk {

// last level: members s_0..s_{K-2}; every extension vertex closes a k-set
template <int K, int V>
__device__ __forceinline__ void leaf(EnumState<K, V> &s, const int (&st)[K - 1], uint32_t code)
{
    const int lane = lane_id();
    int rem[K - 1];
    int total = 0;
#pragma unroll
    for (int q = 0; q < K - 1; ++q) {
        rem[q] = s.len[q] - st[q];
        total += rem[q];
    }
    for (int base = 0; base < total; base += kWave) {
        int a = base + lane;
        const bool valid = a < total;
        int addr = 0;
        bool found = false;
#pragma unroll
        for (int q = 0; q < K - 1; ++q) {
            if (!found) {
                if (a < rem[q]) {
                    addr = q * s.seg_cap + st[q] + a;
                    found = true;
                } else {
                    a -= rem[q];
                }
            }
        }
        uint32_t c = 0;
        if (valid) {
            const uint32_t u = s.seg[addr];
            c = code | code_bits<K>(s.mark[u], K - 1);
        }
        count_codes<K>(s, valid, c);
    }
}


// Position in seg storage of element a of an extension list made of the
// tails seg[q][st[q]:] (rem[q] elements each), q < NQ.
template <int K, int NQ, int V>
__device__ __forceinline__ int ext_addr(const EnumState<K, V> &s, const int (&st)[K - 1],
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

// two-bit relation of w to u: bit0 arc w -> u, bit1 arc u -> w
template <int K, int V>
__device__ __forceinline__ uint32_t pair_type(const EnumState<K, V> &s, uint32_t w, uint32_t u)
{
    if constexpr ((V & kVarSearch) != 0) {
        return list_relation(s.urow, s.uadj, w, u);
    } else {
        const size_t word = (size_t)w * s.words + (u >> 5);
        const uint32_t sh = u & 31u;
        return ((s.bits_out[word] >> sh) & 1u) | (((s.bits_in[word] >> sh) & 1u) << 1);
    }
}


// lane l's value of v (ds_bpermute).  Call with every lane active: a
// permute reads 0 from a lane that is masked off.
__device__ __forceinline__ uint32_t from_lane(uint32_t v, int l)
{
    return (uint32_t)__builtin_amdgcn_ds_bpermute(l << 2, (int)v);
}

// last_two for an extension list that fits one wavefront and children
// jlo..e-1: lane l holds E[l] with its code bits for positions k-2 and k-1
// and its list row, so pair and neighbour items fetch them with one lane
// permute each; pairs and neighbours share wave iterations.
template <int K, int V>
__device__ void last_two_small(EnumState<K, V> &s, const int (&st)[K - 1],
                               const int (&rem)[K - 2], int e, uint32_t code, int jlo)
{
    constexpr int NQ = K - 2;
    constexpr int P1 = K - 2, P2 = K - 1;
    constexpr int B_WU = (K - 2) * (K - 1) + (K - 2);
    constexpr int B_UW = (K - 1) * (K - 1) + (K - 2);
    const int lane = lane_id();
    uint32_t vtx = 0, cb1 = 0, cb2 = 0;
    int row = 0, deg = 0;
    if (lane < e) {
        vtx = s.seg[ext_addr<K, NQ>(s, st, rem, lane)];
        const uint32_t m = s.mark[vtx];
        cb1 = code_bits<K>(m, P1);
        cb2 = code_bits<K>(m, P2);
        row = s.urow[vtx];
        deg = s.urow[vtx + 1] - row;
    }
    if (lane < jlo) deg = 0;
    // children with long lists alone: only the arc type varies
    unsigned long long big = __ballot(deg >= kRowMin);
    while (big) {
        const int l = __builtin_ctzll(big);
        big &= big - 1;
        const int brow = __builtin_amdgcn_readlane(row, l);
        const int bdeg = __builtin_amdgcn_readlane(deg, l);
        const uint32_t bcode = code | (uint32_t)__builtin_amdgcn_readlane((int)cb1, l);
        uint32_t n1 = 0, n2 = 0, n3 = 0;
        for (int b = 0; b < bdeg; b += kWave) {
            const int e2 = b + lane;
            uint32_t t = 0;
            if (e2 < bdeg) {
                const uint32_t ent = s.uadj[brow + e2];
                const int u = (int)(ent >> 2);
                if (u > s.root && s.mark[u] == 0u) t = ent & 3u;
            }
            n1 += (uint32_t)__popcll(__ballot(t == 1u));
            n2 += (uint32_t)__popcll(__ballot(t == 2u));
            n3 += (uint32_t)__popcll(__ballot(t == 3u));
        }
        const uint32_t tl = (uint32_t)lane + 1u;
        const uint32_t nl = lane == 0 ? n1 : (lane == 1 ? n2 : n3);
        s.hpending += n1 + n2 + n3;
        hash_insert<K>(s, lane < 3 && nl > 0, bcode | ((tl & 1u) << B_WU) | ((tl >> 1) << B_UW), nl);
    }
    if (deg >= kRowMin) deg = 0;
    int incl = deg;
    incl = wave_incl_sum(incl);
    const int totB = __builtin_amdgcn_readlane(incl, kWave - 1);
    uint32_t *pre = s.scratch;  // flat_source's buffer
    // flat entry f of this lane's list sits at rowb + f
    const int rowb = row - (incl - deg);
    const int mm = e - jlo;
    const int npairs = mm * (mm - 1) / 2;
    const int total = npairs + totB;
    for (int base = 0; base < total; base += kWave) {
        const int f = base + lane;
        bool valid = f < total;
        const bool pair = f < npairs;
        // source lanes first; the permutes run with every lane active (a
        // permute from an inactive lane reads 0)
        const int srcB = base + kWave > npairs ? flat_source(pre, incl, deg, base - npairs) : 0;
        int src1 = 0, src2 = 0, off = 0;
        if (pair) {
            int b = (int)((1.0f + __builtin_amdgcn_sqrtf(1.0f + 8.0f * (float)f)) * 0.5f);
            b -= (b * (b - 1) / 2 > f) ? 1 : 0;
            b += ((b + 1) * b / 2 <= f) ? 1 : 0;
            src1 = jlo + (f - b * (b - 1) / 2);
            src2 = jlo + b;
        } else if (valid) {
            src1 = srcB;
            off = f - npairs;
        }
        const uint32_t w = from_lane(vtx, src1);
        const uint32_t u2 = from_lane(vtx, src2);
        const uint32_t c1 = from_lane(cb1, src1);
        const uint32_t c2 = from_lane(cb2, src2);
        const int r1 = (int)from_lane((uint32_t)rowb, src1);
        uint32_t c = 0;
        if (pair) {
            const uint32_t t = pair_type<K>(s, w, u2);
            c = code | c1 | c2 | ((t & 1u) << B_WU) | ((t >> 1) << B_UW);
        } else if (valid) {
            const uint32_t ent = s.uadj[r1 + off];
            const int u = (int)(ent >> 2);
            const uint32_t t = ent & 3u;
            valid = u > s.root && s.mark[u] == 0u;
            c = code | c1 | ((t & 1u) << B_WU) | ((t >> 1) << B_UW);
        }
        count_codes<K>(s, valid, c);
    }
    __syncthreads();
}

// Nodes with at most one wave of extension vertices, when marks are 32-bit
// (k = 6, and every k with marks in device memory): the pairs inside E are
// counted per pair of cells, as in Section 3's loop over L_{k-2}, with no
// arc test between two extension vertices.  Two
// vertices with equal marks relate alike to the members, so all pairs of E
// from cells A and B without an arc between them have one code; there are
// C(n_A, 2) or n_A n_B of them.  The arcs inside E are found while the
// children's lists are scanned for Part B: E's vertices carry kETag and
// their lane in their (32-bit) marks meanwhile, and each arc (w, u), u
// after w, adds one to its own code and takes one from its cell pair's.
// Part B is counted as in last_two_small.
constexpr uint32_t kETag = 1u << 30;  // mark bits 24..29: the vertex's lane

template <int K, int V>
__device__ void last_two_cells(EnumState<K, V> &s, const int (&st)[K - 1],
                               const int (&rem)[K - 2], int e, uint32_t code, int jlo)
{
    static_assert(sizeof(MarkT<K, V>) == 4, "E tags need 32-bit marks");
    constexpr int NQ = K - 2;
    constexpr int P1 = K - 2, P2 = K - 1;
    constexpr int B_WU = (K - 2) * (K - 1) + (K - 2);
    constexpr int B_UW = (K - 1) * (K - 1) + (K - 2);
    const int lane = lane_id();
    const bool inE = lane >= jlo && lane < e;
    uint32_t vtx = 0, cb1 = 0, cb2 = 0, m0 = 0;
    int row = 0, deg = 0;
    if (lane < e) {
        vtx = s.seg[ext_addr<K, NQ>(s, st, rem, lane)];
        m0 = s.mark[vtx];
        cb1 = code_bits<K>(m0, P1);
        cb2 = code_bits<K>(m0, P2);
        row = s.urow[vtx];
        deg = s.urow[vtx + 1] - row;
    }
    if (!inE) deg = 0;
    if (inE) s.mark[vtx] = (MarkT<K, V>)(m0 | kETag | ((uint32_t)lane << 24));
    __syncthreads();
    auto tbits = [](uint32_t t) { return ((t & 1u) << B_WU) | ((t >> 1) << B_UW); };

    // children with long lists alone: exclusive neighbours by type, arcs to
    // later vertices of E one by one
    unsigned long long big = __ballot(deg >= kRowMin);
    while (big) {
        const int l = __builtin_ctzll(big);
        big &= big - 1;
        const int brow = __builtin_amdgcn_readlane(row, l);
        const int bdeg = __builtin_amdgcn_readlane(deg, l);
        const uint32_t bcode = code | (uint32_t)__builtin_amdgcn_readlane((int)cb1, l);
        uint32_t n1 = 0, n2 = 0, n3 = 0;
        for (int b = 0; b < bdeg; b += kWave) {
            const int e2 = b + lane;
            uint32_t tb = 0, t = 0;
            bool arc = false;
            int q = 0;
            if (e2 < bdeg) {
                const uint32_t ent = s.uadj[brow + e2];
                const int u = (int)(ent >> 2);
                const uint32_t mu = s.mark[u];
                t = ent & 3u;
                if (mu & kETag) {
                    q = (int)((mu >> 24) & 63u);
                    arc = q > l;
                } else if (u > s.root && mu == 0u) {
                    tb = t;
                }
            }
            n1 += (uint32_t)__popcll(__ballot(tb == 1u));
            n2 += (uint32_t)__popcll(__ballot(tb == 2u));
            n3 += (uint32_t)__popcll(__ballot(tb == 3u));
            const uint32_t cm = bcode | from_lane(cb2, q);
            count_codes<K>(s, arc, cm | tbits(t));
            uncount_codes<K>(s, arc, cm);
        }
        const uint32_t tl = (uint32_t)lane + 1u;
        const uint32_t nl = lane == 0 ? n1 : (lane == 1 ? n2 : n3);
        s.hpending += n1 + n2 + n3;
        hash_insert<K>(s, lane < 3 && nl > 0, bcode | tbits(tl), nl);
    }
    if (deg >= kRowMin) deg = 0;
    int incl = deg;
    incl = wave_incl_sum(incl);
    const int totB = __builtin_amdgcn_readlane(incl, kWave - 1);
    uint32_t *pre = s.scratch;  // flat_source's buffer
    // flat entry f of this lane's list sits at rowb + f
    const int rowb = row - (incl - deg);
    // the short lists, flat: Part B entries and arcs inside E
    for (int base = 0; base < totB; base += kWave) {
        const int f = base + lane;
        const bool valid = f < totB;
        const int src1 = flat_source(pre, incl, deg, base);
        const int off = f;
        // the permutes run with every lane active
        const int r1 = (int)from_lane((uint32_t)rowb, src1);
        const uint32_t c1 = from_lane(cb1, src1);
        bool bv = false, arc = false;
        uint32_t t = 0;
        int q = 0;
        if (valid) {
            const uint32_t ent = s.uadj[r1 + off];
            const int u = (int)(ent >> 2);
            const uint32_t mu = s.mark[u];
            t = ent & 3u;
            if (mu & kETag) {
                q = (int)((mu >> 24) & 63u);
                arc = q > src1;
            } else {
                bv = u > s.root && mu == 0u;
            }
        }
        const uint32_t cm = code | c1 | from_lane(cb2, q);
        count_codes<K>(s, bv, code | c1 | tbits(t));
        count_codes<K>(s, arc, cm | tbits(t));
        uncount_codes<K>(s, arc, cm);
    }
    __syncthreads();

    // the cells of E (vertices with equal marks) and their pairs
    const uint32_t key = inE ? cb1 : 0xFFFFFFFFu;
    unsigned long long left = __ballot(inE);
    bool leader = false;
    uint32_t size = 0;
    while (left) {
        const int l = __builtin_ctzll(left);
        const uint32_t k0 = (uint32_t)__builtin_amdgcn_readlane((int)key, l);
        const unsigned long long eq = __ballot(key == k0) & left;
        if (lane == l) {
            leader = true;
            size = (uint32_t)__popcll(eq);
        }
        left &= ~eq;
    }
    const unsigned long long leaders = __ballot(leader);
    const int ncell = __popcll(leaders);
    uint32_t *cc1 = s.scratch + kWave, *cc2 = s.scratch + 2 * kWave;
    if (leader) {
        const int rk = (int)lanes_below(leaders);
        cc1[rk] = cb1 | (size << 24);  // cb1 < 2^24 for k <= 6
        cc2[rk] = cb2;
    }
    __syncthreads();
    const int mm = e - jlo;
    const uint32_t all_pairs = (uint32_t)(mm * (mm - 1) / 2);
    if (s.hpending + all_pairs >= kPendingMax) flush_hash<K>(s);
    s.hpending += all_pairs;
    const int ncp = ncell * (ncell + 1) / 2;
    for (int pb = 0; pb < ncp; pb += kWave) {
        const int p = pb + lane;
        bool valid = p < ncp;
        uint32_t c = 0, w = 0;
        if (valid) {
            // p = z(z+1)/2 + y with y <= z
            int z = (int)((__builtin_amdgcn_sqrtf(8.0f * (float)p + 1.0f) - 1.0f) * 0.5f);
            if ((z + 1) * (z + 2) / 2 <= p) ++z;
            if (z * (z + 1) / 2 > p) --z;
            const int y = p - z * (z + 1) / 2;
            const uint32_t xy = cc1[y], xz = cc1[z];
            const uint32_t ny = xy >> 24, nz = xz >> 24;
            w = y == z ? ny * (ny - 1u) / 2u : ny * nz;
            c = code | (xy & 0xFFFFFFu) | cc2[z];
            valid = w > 0u;
        }
        hash_insert<K>(s, valid, c, w);
    }
    if (inE) s.mark[vtx] = (MarkT<K, V>)m0;
    __syncthreads();
}

// The last two ESU levels of a node X with k-2 members s_0..s_{k-3} and
// extension list E, done flat across the wavefront without adding members.
// Child w = E[i] (i in [jlo, jhi)) closes the k-sets X + {w, u} for
//   (A) u = E[j], j > i: w's and u's relations to X come from their marks,
//       the relation between w and u from the adjacency bit matrices (the
//       pair test of Algorithm 2, Section 3.1);
//   (B) u an exclusive neighbour of w (u > root, mark[u] == 0): u has no arc
//       to X, its relation to w is the type of the entry in w's list (the
//       neighbour-list scan of Algorithm 3).
// (A) and (B) together are exactly ESU's extension list of the child w.
template <int K, int V>
__device__ void last_two(EnumState<K, V> &s, const int (&st)[K - 1], uint32_t code, int jlo, int jhi)
{
    constexpr int NQ = K - 2;
    constexpr int P1 = K - 2, P2 = K - 1;
    constexpr int B_WU = (K - 2) * (K - 1) + (K - 2);  // bit of arc s_{k-2} -> s_{k-1}
    constexpr int B_UW = (K - 1) * (K - 1) + (K - 2);  // bit of arc s_{k-1} -> s_{k-2}
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
        if constexpr (sizeof(MarkT<K, V>) == 4) last_two_cells<K>(s, st, rem, e, code, jlo);
        else last_two_small<K>(s, st, rem, e, code, jlo);
        return;
    }

    // (A) pairs (E[i], E[j]), j > i.  Long rows run one at a time with the
    // row's vertex w wave-uniform; the short rows left at the end run flat.
    int i0 = jlo;
    for (; i0 < hi && e - 1 - i0 >= kRowMin; ++i0) {
        const uint32_t w = (uint32_t)uniform((int)s.seg[ext_addr<K, NQ>(s, st, rem, i0)]);
        const uint32_t cw = code | code_bits<K>((uint32_t)uniform((int)s.mark[w]), P1);
        const size_t wrow = (V & kVarSearch) != 0 ? 0 : (size_t)w * s.words;
        for (int jb = i0 + 1; jb < e; jb += kWave) {
            const int j = jb + lane;
            const bool valid = j < e;
            uint32_t c = 0;
            if (valid) {
                const uint32_t u = s.seg[ext_addr<K, NQ>(s, st, rem, j)];
                uint32_t t;
                if constexpr ((V & kVarSearch) != 0) {
                    t = list_relation(s.urow, s.uadj, w, u);
                } else {
                    const uint32_t sh = u & 31u;
                    t = ((s.bits_out[wrow + (u >> 5)] >> sh) & 1u) |
                        (((s.bits_in[wrow + (u >> 5)] >> sh) & 1u) << 1);
                }
                c = cw | code_bits<K>(s.mark[u], P2) | ((t & 1u) << B_WU) | ((t >> 1) << B_UW);
            }
            count_codes<K>(s, valid, c);
        }
    }
    // flat: the short rows left, i0 <= i < hi.  When they run to the end
    // of E the pairs form the triangle a < b < m over E[i0..e) (m <= kRowMin),
    // taken in b-major order: b = floor((1 + sqrt(1 + 8p)) / 2),
    // a = p - b(b-1)/2.  Otherwise (a range-limited unit) row by row.
    const int m = e - i0;
    const bool tri = hi == e;
    const int A = e - 1 - i0;
    const int rows = hi - i0;
    const int npairs = rows <= 0 ? 0 : (tri ? m * (m - 1) / 2 : rows * A - rows * (rows - 1) / 2);
    const float tA = 2.0f * (float)A + 1.0f;
    for (int base = 0; base < npairs; base += kWave) {
        const int p = base + lane;
        const bool valid = p < npairs;
        uint32_t c = 0;
        if (valid) {
            int i, j;
            if (tri) {
                int b = (int)((1.0f + __builtin_amdgcn_sqrtf(1.0f + 8.0f * (float)p)) * 0.5f);
                b -= (b * (b - 1) / 2 > p) ? 1 : 0;
                b += ((b + 1) * b / 2 <= p) ? 1 : 0;
                i = i0 + (p - b * (b - 1) / 2);
                j = i0 + b;
            } else {
                float disc = tA * tA - 8.0f * (float)p;
                disc = disc > 0.f ? disc : 0.f;
                int r = (int)((tA - __builtin_amdgcn_sqrtf(disc)) * 0.5f);
                r = r < 0 ? 0 : (r > rows - 1 ? rows - 1 : r);
                while (r + 1 < rows && (r + 1) * A - (r + 1) * r / 2 <= p) ++r;
                while (r > 0 && r * A - r * (r - 1) / 2 > p) --r;
                i = i0 + r;
                j = i + 1 + (p - (r * A - r * (r - 1) / 2));
            }
            if (i < j && j < e) {
                const uint32_t w = s.seg[ext_addr<K, NQ>(s, st, rem, i)];
                const uint32_t u = s.seg[ext_addr<K, NQ>(s, st, rem, j)];
                const uint32_t t = pair_type<K>(s, w, u);
                c = code | code_bits<K>(s.mark[w], P1) | code_bits<K>(s.mark[u], P2) |
                    ((t & 1u) << B_WU) | ((t >> 1) << B_UW);
            } else {
                atomicAdd(s.errors, 1u);  // unreachable: the decode keeps i < j < e
            }
        }
        count_codes<K>(s, valid && c != 0, c);
    }

    // (B) exclusive neighbours, 64 children at a time.  A child of degree
    // >= kRowMin is scanned alone: its new neighbours all have mark 0, so
    // only the arc type varies and three scalar counts carry the result.
    // The others run flat, a lane-prefix sum of their degrees mapping a flat
    // index to (child, list position).
    uint32_t *pre = s.scratch, *start = s.scratch + kWave, *cw = s.scratch + 2 * kWave;
    for (int ib = jlo; ib < hi; ib += kWave) {
        const int i = ib + lane;
        int deg = 0, row = 0;
        uint32_t wcode = 0;
        if (i < hi) {
            const uint32_t w = s.seg[ext_addr<K, NQ>(s, st, rem, i)];
            row = s.urow[w];
            deg = s.urow[w + 1] - row;
            wcode = code_bits<K>(s.mark[w], P1);
        }
        unsigned long long big = __ballot(deg >= kRowMin);
        while (big) {
            const int l = __builtin_ctzll(big);
            big &= big - 1;
            const int brow = __builtin_amdgcn_readlane(row, l);
            const int bdeg = __builtin_amdgcn_readlane(deg, l);
            const uint32_t bcode = code | (uint32_t)__builtin_amdgcn_readlane((int)wcode, l);
            uint32_t n1 = 0, n2 = 0, n3 = 0;
            for (int b = 0; b < bdeg; b += kWave) {
                const int e2 = b + lane;
                uint32_t t = 0;
                if (e2 < bdeg) {
                    const uint32_t ent = s.uadj[brow + e2];
                    const int u = (int)(ent >> 2);
                    if (u > s.root && s.mark[u] == 0u) t = ent & 3u;
                }
                n1 += (uint32_t)__popcll(__ballot(t == 1u));
                n2 += (uint32_t)__popcll(__ballot(t == 2u));
                n3 += (uint32_t)__popcll(__ballot(t == 3u));
            }
            const uint32_t tl = (uint32_t)lane + 1u;
            const uint32_t nl = lane == 0 ? n1 : (lane == 1 ? n2 : n3);
            s.hpending += n1 + n2 + n3;
            hash_insert<K>(s, lane < 3 && nl > 0, bcode | ((tl & 1u) << B_WU) | ((tl >> 1) << B_UW), nl);
        }
        if (deg >= kRowMin) deg = 0;
        int incl = deg;
        incl = wave_incl_sum(incl);
        const int tot = __builtin_amdgcn_readlane(incl, kWave - 1);
        start[lane] = (uint32_t)(row - (incl - deg));  // flat entry f at start + f
        cw[lane] = wcode;
        __syncthreads();
        for (int fb = 0; fb < tot; fb += kWave) {
            const int f = fb + lane;
            bool valid = f < tot;
            uint32_t c = 0;
            const int lo = flat_source(pre, incl, deg, fb);
            if (valid) {
                const uint32_t ent = s.uadj[start[lo] + (uint32_t)f];
                const int u = (int)(ent >> 2);
                const uint32_t t = ent & 3u;
                valid = u > s.root && s.mark[u] == 0u;
                c = code | cw[lo] | ((t & 1u) << B_WU) | ((t >> 1) << B_UW);
            }
            count_codes<K>(s, valid, c);
        }
        __syncthreads();
    }
}

// node with members s_0..s_D: visit children jlo..jhi-1 of its extension
// list (the tails seg[q][st[q]:] for q <= D, in order)
template <int K, int D, int V>
__device__ void visit(EnumState<K, V> &s, const int (&st)[K - 1], uint32_t code, int jlo, int jhi)
{
    if constexpr (K == 3 && D == 1) {
        leaf<K>(s, st, code);
    } else if constexpr (K >= 4 && D == K - 3) {
        last_two<K>(s, st, code, jlo, jhi);
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
            const uint32_t ccode = code | code_bits<K>(mx, D + 1);
            const Held held = push_held<K, D + 1>(s, x);
            int cst[K - 1];
#pragma unroll
            for (int q = 0; q < K - 1; ++q)
                cst[q] = q < L ? s.len[q] : (q == L ? o + 1 : (q <= D ? st[q] : 0));
            visit<K, D + 1>(s, cst, ccode, 0, INT_MAX);
            pop_held<K, D + 1>(s, x, held);
        }
    }
}

template <int K, int V>
__device__ void run_unit(EnumState<K, V> &s, int v, int i, uint32_t range)
{
    s.root = v;
    const Held held0 = push_held<K, 0>(s, v);
    if (i < s.len[0]) {
        const int x = uniform((int)s.seg[i]);
        const uint32_t code = code_bits<K>((uint32_t)uniform((int)s.mark[x]), 1);
        const Held held1 = push_held<K, 1>(s, x);
        int st[K - 1];
#pragma unroll
        for (int q = 0; q < K - 1; ++q) st[q] = 0;
        st[0] = i + 1;
        const bool full = range == kFullChild;
        visit<K, 1>(s, st, code, full ? 0 : (int)(range & 0xFFFFu), full ? INT_MAX : (int)(range >> 16));
        pop_held<K, 1>(s, x, held1);
    } else if (lane_id() == 0) {
        atomicAdd(s.errors, 1u);
    }
    pop_held<K, 0>(s, v, held0);
}

template <int K, int V>
__device__ __forceinline__ void enum_body(const DevGraph *graphs, const int4 *units,
                                          uint32_t unit_cap, uint32_t unit_end, uint32_t *counters,
                                          const uint32_t *table, uint32_t num_classes,
                                          unsigned long long *hist_base, const EnumConfig &cfg)
{
    extern __shared__ uint32_t lds[];
    EnumState<K, V> s;
    const LdsLayout lay = lds_layout(K, cfg.max_n, cfg.seg_cap, cfg.hash_bits, (V & kVarGlobal) != 0);
    init_state(s, reinterpret_cast<char *>(lds), lay, cfg, counters, table, num_classes);
    for_each_unit<false, K>(s, graphs, units, unit_cap, unit_end, counters, hist_base, cfg,
                     [&](int v, int i, uint32_t range) { run_unit<K>(s, v, i, range); });
}

// bit-matrix arc tests, LDS marks
template <int K>
__global__ __launch_bounds__(kWave) void enum_kernel(const DevGraph *graphs, const int4 *units,
                                                     uint32_t unit_cap, uint32_t unit_end,
                                                     uint32_t *counters,
                                                     const uint32_t *table, uint32_t num_classes,
                                                     unsigned long long *hist_base,
                                                     EnumConfig cfg)
{
    enum_body<K, 0>(graphs, units, unit_cap, unit_end, counters, table, num_classes, hist_base, cfg);
}

// the test-hook builds of the variants above (V includes kVarDebug)
template <int K, int V>
__global__ __launch_bounds__(kWave) void enum_debug_kernel(const DevGraph *graphs, const int4 *units,
                                                           uint32_t unit_cap, uint32_t unit_end,
                                                           uint32_t *counters,
                                                           const uint32_t *table, uint32_t num_classes,
                                                           unsigned long long *hist_base,
                                                           EnumConfig cfg)
{
    enum_body<K, V>(graphs, units, unit_cap, unit_end, counters, table, num_classes, hist_base, cfg);
}

// arc tests by list search (V = kVarSearch, optionally | kVarGlobal)
template <int K, int V>
__global__ __launch_bounds__(kWave) void enum_lists_kernel(const DevGraph *graphs, const int4 *units,
                                                           uint32_t unit_cap, uint32_t unit_end,
                                                           uint32_t *counters,
                                                           const uint32_t *table, uint32_t num_classes,
                                                           unsigned long long *hist_base,
                                                           EnumConfig cfg)
{
    enum_body<K, V>(graphs, units, unit_cap, unit_end, counters, table, num_classes, hist_base, cfg);
}

int enum_hash_bits(int) { return kHashBits; }

int enum_lds_bytes(int k, int max_n, int seg_cap, int variant)
{
    return lds_layout(k, max_n, seg_cap, enum_hash_bits(k), (variant & kVarGlobal) != 0).total;
}

// the instantiated variants: bit matrices, list search, list search with
// global marks; each also with the test hooks
template <int K>
static const void *enum_fn(int variant)
{
    switch (variant) {
    case 0: return reinterpret_cast<const void *>(&enum_kernel<K>);
    case kVarSearch: return reinterpret_cast<const void *>(&enum_lists_kernel<K, kVarSearch>);
    case kVarSearch | kVarGlobal:
        return reinterpret_cast<const void *>(&enum_lists_kernel<K, kVarSearch | kVarGlobal>);
    case kVarDebug: return reinterpret_cast<const void *>(&enum_debug_kernel<K, kVarDebug>);
    case kVarDebug | kVarSearch:
        return reinterpret_cast<const void *>(&enum_debug_kernel<K, kVarDebug | kVarSearch>);
    case kVarDebug | kVarSearch | kVarGlobal:
        return reinterpret_cast<const void *>(
            &enum_debug_kernel<K, kVarDebug | kVarSearch | kVarGlobal>);
    default: return nullptr;
    }
}

static const void *enum_fn(int k, int variant)
{
    switch (k) {
    case 3: return enum_fn<3>(variant);
    case 4: return enum_fn<4>(variant);
    case 5: return enum_fn<5>(variant);
    case 6: return enum_fn<6>(variant);
    default: return nullptr;
    }
}

int enum_max_blocks_per_cu(int k, int variant, int lds_bytes, int *blocks)
{
    const void *fn = enum_fn(k, variant);
    if (!fn) return fail(MK_ERANGE, "no enumeration kernel for k=%d, variant %d", k, variant);
    MK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, fn, kWave, (size_t)lds_bytes));
    return MK_OK;
}

int launch_enum(int k, const DevGraph *d_graphs, const int4 *units, uint32_t unit_cap,
                uint32_t unit_end, uint32_t *counters, const uint32_t *table, uint32_t num_classes,
                unsigned long long *hist_base, const EnumConfig &cfg, int grid, int lds_bytes,
                hipStream_t stream)
{
    if (grid <= 0) return MK_OK;
    const void *fn = enum_fn(k, cfg.variant);
    if (!fn) return fail(MK_ERANGE, "no enumeration kernel for k=%d, variant %d", k, cfg.variant);
    if ((cfg.variant & kVarGlobal) != 0 && !cfg.marks)
        return fail(MK_EINVAL, "launch_enum: global marks variant without a marks array");
    EnumConfig c = cfg;
    void *args[] = {(void *)&d_graphs, (void *)&units, (void *)&unit_cap, (void *)&unit_end,
                    (void *)&counters, (void *)&table, (void *)&num_classes, (void *)&hist_base,
                    (void *)&c};
    MK_HIP(hipLaunchKernel(fn, dim3(grid), dim3(kWave), args, (size_t)lds_bytes, stream));
    return MK_OK;
}

}  // namespace mk
