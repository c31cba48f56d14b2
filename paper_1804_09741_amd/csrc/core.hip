// Counting H_k from the connected (k-2)-sets (Section 3, the counting loop
// over L_{k-2}).
//
// A connected (k-2)-set X and any two vertices y, z of adj(X) (the vertices
// outside X with an arc to or from X, Section 2) form a connected k-set.
// Section 2 partitions adj(X) into cells by each vertex's relation (A, B, C
// or none) to every member of X; all vertices of one cell look alike from
// X.  So for two cells Y, Z the k-sets X + {y, z} with no arc between y and z
// all have one class, motif(X, Y, Z), and there are C(|Y|, 2) (Y = Z) or
// |Y| |Z| of them.  Each arc pair u, v inside adj(X) moves one k-set from
// motif(X, cell(u), cell(v)) to the class of G[X + {u, v}].  Summed over X,
// a k-set S is reached once per core of S (a connected (k-2)-subset that both
// other vertices touch); that number depends only on the class of S, so the
// raw sums are divided by it at the end (core_mult of the class table).
//
// Kernel: one 64-lane wave per workgroup, persistent, on the same work
// queues as the enumeration kernel.  The cores X are listed by ESU to depth
// k-2 (the planner runs for (k-1)-sets, so a unit is a range of the nodes
// just above the cores).  The marks that ESU keeps in LDS already hold, for
// every vertex u of adj(X), its relation bits to each member -- its cell --
// and the code bits u adds at any position.  Per core:
//   1. cells: the members' lists are read flat; a vertex is taken from the
//      first member it is adjacent to (no lower member bits in its mark), its
//      cell counted in LDS, new cells appended to a list;
//   2. arcs inside adj(X): the taken vertices' own lists are scanned flat
//      (a lane-prefix sum of degrees); a neighbour v > u with a mark and not
//      a member closes an arc pair.  With few cells the pair is counted in
//      an LDS table per (cell pair, arc type); otherwise it goes straight to
//      the per-wave hash, +1 for the code with the arcs and -1 without;
//   3. cell pairs: lanes take pairs (Y, Z) of the list, form the code of X
//      + one vertex of each (marks expanded back from the cell index) and
//      add the weight, less the table's arc pairs, to the hash; the table's
//      entries go to the codes with their arcs.
// Hash counts are 32-bit two's complement (the -1s); a flush sign-extends
// them into the 64-bit histogram, so partial sums may wrap and the totals
// are exact modulo 2^64 -- which they are, being the final non-negative
// raw counts.
#include "esu.h"

namespace mk {

template <int K>
constexpr int kCoreR = K - 2;                     // members of a core
template <int K>
constexpr int kCells = 1 << (2 * (K - 2));        // 4^(k-2) relation vectors
// The top four bits of a mark (above every relation bit) are all set on
// the members of the core being processed (and of a parent while its arc
// pairs are listed).  Otherwise, on the vertices of adj(X), they hold the
// list position of the vertex's cell (0..14) from the core's cell phase on,
// the arc-pair table's index; they are left as they are until the next
// core overwrites them, or cleared with the vertex's last relation bit.
template <int K>
constexpr int kPosShift = 8 * (int)sizeof(MarkT<K>) - 4;
template <int K>
constexpr uint32_t kMemberFlag = 0xFu << kPosShift<K>;

template <int K>
__device__ __forceinline__ bool is_member(uint32_t m)
{
    return (m & kMemberFlag<K>) == kMemberFlag<K>;
}

// Cores with at most kAggCells cells count their arc pairs in a small LDS
// table per (cell pair, arc type) first; the pair phase then takes them off
// the pair weights and adds them to the true classes, one insert per
// non-empty entry.  Cores with more cells insert +1/-1 per arc pair.
template <int K>
constexpr int kAggCells = K == 6 ? 12 : 15;
template <int K>
constexpr int kAggWords = 3 * kAggCells<K> * (kAggCells<K> + 1) / 2;

// Extension segments the core walk fills: those of members 0..k-4 (a
// core's last member only marks).
template <int K>
constexpr int kCoreSegs = K - 3;
// The arc scan keeps each of its 64 vertices' id beside its mark: in one
// word while marks are 16-bit (k <= 5; LDS marks mean ids below 8,192, in
// the high half), else in 64 words of their own.
template <int K>
constexpr bool kPackedUid = sizeof(MarkT<K>) == 2;

// LDS of the core kernel beyond the enumeration layout: cell counts (u32),
// the list of non-empty cells and each cell's list position (u8), the arc
// scan's vertex ids (k = 6), and the arc-pair table.  A wave's LDS sets how
// many waves a CU holds, and the kernel's speed follows that count.
struct CoreLds {
    uint32_t *cnt;
    uint8_t *list;
    uint8_t *pos;
    uint32_t *uid;  // null when packed with the marks
    uint32_t *agg;
    uint32_t *ap;  // global: this workgroup's arc list of the current parent
};

__host__ __device__ inline int core_extra_bytes(int k)
{
    const int cells = 1 << (2 * (k - 2));
    const int agg_cells = k == 6 ? 12 : 15;
    return 4 * cells + 2 * ((cells + 3) & ~3) + (k >= 6 ? 4 * kWave : 0) +
           4 * 3 * agg_cells * (agg_cells + 1) / 2;
}

// relation vector of a mark: bits 0..R-1 = arcs u -> s_0..s_{R-1} (the
// mark's out bits, already adjacent), bits R..2R-1 = arcs s_0..s_{R-1} -> u
// (its in bits, at stride k-1)
template <int K>
__device__ __forceinline__ uint32_t cell_of(uint32_t m)
{
    constexpr int R = kCoreR<K>;
    uint32_t c = (m >> EnumState<K>::OUTB) & ((1u << R) - 1u);
#pragma unroll
    for (int d = 0; d < R; ++d) c |= ((m >> (d * (K - 1))) & 1u) << (R + d);
    return c;
}

// inverse of cell_of
template <int K>
__device__ __forceinline__ uint32_t mark_of_cell(uint32_t c)
{
    constexpr int R = kCoreR<K>;
    uint32_t m = (c & ((1u << R) - 1u)) << EnumState<K>::OUTB;
#pragma unroll
    for (int d = 0; d < R; ++d) m |= ((c >> (R + d)) & 1u) << (d * (K - 1));
    return m;
}

// mark bits of member positions below d
template <int K>
__device__ __forceinline__ uint32_t lower_members(int d)
{
    uint32_t m = 0;
#pragma unroll
    for (int q = 0; q < kCoreR<K>; ++q)
        if (q < d) m |= (1u << (q * (K - 1))) | (1u << (EnumState<K>::OUTB + q));
    return m;
}

// s_D := x for the last member of a core: marks only (no extension segment)
template <int K, int D, int V>
__device__ __forceinline__ void push_marks(EnumState<K, V> &s, int x)
{
    const int lane = lane_id();
    const int r0 = uniform(s.urow[x]);
    const int r1 = uniform(s.urow[x + 1]);
    for (int base = r0; base < r1; base += kWave) {
        const int e = base + lane;
        if (e < r1) {
            const uint32_t ent = s.uadj[e];
            const int y = (int)(ent >> 2);
            s.mark[y] = (MarkT<K>)(s.mark[y] | mark_bits<K>(D, ent & 3u));
        }
    }
    __syncthreads();
}

// push_marks<D>(x) keeping the list for pop_held (see push_held)
template <int K, int D, int V>
__device__ __forceinline__ Held push_marks_held(EnumState<K, V> &s, int x)
{
    const int lane = lane_id();
    const int r0 = uniform(s.urow[x]);
    const int r1 = uniform(s.urow[x + 1]);
    Held h;
    h.n = r1 - r0;
    h.ent = 0u;
    h.m = 0u;
    if (h.n > kWave) {
        push_marks<K, D>(s, x);
        return h;
    }
    if (lane < h.n) {
        h.ent = s.uadj[r0 + lane];
        const int y = (int)(h.ent >> 2);
        h.m = s.mark[y];
        s.mark[y] = (MarkT<K>)(h.m | mark_bits<K>(D, h.ent & 3u));
    }
    __syncthreads();
    return h;
}

// pop_held<D>(x) for the core walk: a long list's pop also clears the
// position bits of the vertices it leaves without any relation bit (a short
// list's pop restores the marks from before the push, where a vertex
// without relation bits had no position bits either)
template <int K, int D, int V>
__device__ __forceinline__ void core_pop(EnumState<K, V> &s, int x, const Held &h)
{
    if (h.n <= kWave) {
        pop_held<K, D>(s, x, h);
        return;
    }
    const int lane = lane_id();
    const int r0 = uniform(s.urow[x]);
    const int r1 = uniform(s.urow[x + 1]);
    const uint32_t keep = ~mark_bits<K>(D, 3u);
    for (int base = r0; base < r1; base += kWave) {
        const int e = base + lane;
        if (e < r1) {
            const int y = (int)(s.uadj[e] >> 2);
            uint32_t m = s.mark[y] & keep;
            if (!(m & ~kMemberFlag<K>)) m = 0u;
            s.mark[y] = (MarkT<K, V>)m;
        }
    }
    __syncthreads();
}

// Class id of a code for the class-keyed hash of the core kernel (cores
// stand for many differently labelled k-sets, so their codes rarely repeat
// while their classes do).  A code outside the connected classes is a
// device error and is dropped.
template <int K, int V>
__device__ __forceinline__ uint32_t class_of(EnumState<K, V> &s, bool &valid, uint32_t code)
{
    uint32_t id = 0;
    if (valid) {
        id = s.table[code];
        if (id >= s.num_classes) {
            atomicAdd(s.errors, 1u);
            valid = false;
        }
    }
    return id;
}

// Flat index a over the concatenated lists of the members: member d and
// list position e.
template <int R>
__device__ __forceinline__ int member_entry(const int (&pre)[R + 1], const int (&r0)[R], int a,
                                            int *d)
{
    int dd = 0;
#pragma unroll
    for (int q = 1; q < R; ++q) dd += a >= pre[q] ? 1 : 0;
    int e = 0;
#pragma unroll
    for (int q = 0; q < R; ++q)
        if (q == dd) e = r0[q] + (a - pre[q]);
    *d = dd;
    return e;
}

// Flat scan over the vertices u taken from the lists of members
// from..NM-1 (first-seen -- no mark bits of a lower member -- and not a
// member): every entry of u's own list is handed to
// arc(edge, u, v, mark u, mark v, arc type), edge = v has a mark, is not a
// member, and keep(v, u, mark v).  Padding lanes get edge = false.
template <int K, int NM, int V, typename Keep, typename Arc>
__device__ __forceinline__ void scan_taken(EnumState<K, V> &s, const CoreLds &c,
                                           const int (&pre)[NM + 1], const int (&r0)[NM],
                                           int from, Keep keep, Arc arc)
{
    constexpr uint32_t FLAG = kMemberFlag<K>;
    const int lane = lane_id();
    uint32_t *srcb = s.scratch, *start = s.scratch + kWave, *cw = s.scratch + 2 * kWave;
    for (int base = pre[from]; base < pre[NM]; base += kWave) {
        const int a = base + lane;
        int deg = 0, row = 0, u = 0;
        uint32_t mu = 0;
        if (a < pre[NM]) {
            int d;
            const int e = member_entry<NM>(pre, r0, a, &d);
            u = (int)(s.uadj[e] >> 2);
            const uint32_t m = s.mark[u];
            if (!is_member<K>(m) && !(m & lower_members<K>(d))) {
                row = s.urow[u];
                deg = s.urow[u + 1] - row;
                mu = m;
            }
        }
        int incl = deg;
        incl = wave_incl_sum(incl);
        const int tot = __builtin_amdgcn_readlane(incl, kWave - 1);
        start[lane] = (uint32_t)(row - (incl - deg));  // flat entry f at start + f
        if constexpr (kPackedUid<K>) {
            cw[lane] = mu | ((uint32_t)u << 16);
        } else {
            cw[lane] = mu;
            c.uid[lane] = (uint32_t)u;
        }
        __syncthreads();
        for (int fb = 0; fb < tot; fb += kWave) {
            const int f = fb + lane;
            bool edge = false;
            int uu = 0, v = 0;
            uint32_t m_u = 0, mv = 0, t = 0;
            const int lo = flat_source(srcb, incl, deg, fb);
            if (f < tot) {
                const uint32_t ent = s.uadj[start[lo] + (uint32_t)f];
                v = (int)(ent >> 2);
                mv = s.mark[v];
                const uint32_t w = cw[lo];
                if constexpr (kPackedUid<K>) {
                    uu = (int)(w >> 16);
                    m_u = w & 0xFFFFu;
                } else {
                    uu = (int)c.uid[lo];
                    m_u = w;
                }
                t = ent & 3u;
                edge = mv != 0u && !is_member<K>(mv) && keep(v, uu, mv);
            }
            arc(edge, uu, v, m_u, mv, t);
        }
        __syncthreads();
    }
}

// The arc pairs (u, v), u < v, inside adj(P) for the parent P = mem[0..NP-1]
// (all pushed, nothing below): into c.ap as u | v << 13 | type << 26.
// Returns their number, or -1 when they exceed kParentArcCap.
template <int K, int NP, int V>
__device__ int parent_arcs(EnumState<K, V> &s, const CoreLds &c, const int (&mem)[K])
{
    constexpr uint32_t FLAG = kMemberFlag<K>;
    const int lane = lane_id();
#pragma unroll
    for (int d = 0; d < NP; ++d)
        if (lane == d) s.mark[mem[d]] = (MarkT<K>)(s.mark[mem[d]] | FLAG);
    int r0[NP], pre[NP + 1];
    pre[0] = 0;
#pragma unroll
    for (int d = 0; d < NP; ++d) {
        r0[d] = uniform(s.urow[mem[d]]);
        pre[d + 1] = pre[d] + uniform(s.urow[mem[d] + 1]) - r0[d];
    }
    __syncthreads();
    int nap = 0;
    scan_taken<K, NP>(
        s, c, pre, r0, 0, [](int v, int u, uint32_t) { return v > u; },
        [&](bool edge, int u, int v, uint32_t, uint32_t, uint32_t t) {
            const unsigned long long bal = __ballot(edge);
            const int at = nap + (int)lanes_below(bal);
            if (edge && at < (int)kParentArcCap)
                c.ap[at] = (uint32_t)u | ((uint32_t)v << 13) | (t << 26);
            nap += __popcll(bal);
        });
#pragma unroll
    for (int d = 0; d < NP; ++d)
        if (lane == d) s.mark[mem[d]] = (MarkT<K>)(s.mark[mem[d]] & ~FLAG);
    __syncthreads();
    return nap > (int)kParentArcCap ? -1 : nap;
}

// one core X = mem[0..k-3] with internal code cx (all members pushed)
// nap >= 0: c.ap holds the nap arc pairs inside adj(P), P = X less its last
// member z, so only the vertices z brings have their lists scanned; nap < 0:
// every taken vertex's list is scanned.
template <int K, int V>
__device__ void core_node(EnumState<K, V> &s, const CoreLds &c, const int (&mem)[K], uint32_t cx,
                          int nap)
{
    constexpr int R = kCoreR<K>;
    constexpr uint32_t FLAG = kMemberFlag<K>;
    // arc bits between positions k-2 and k-1
    constexpr int B_YZ = (K - 2) * (K - 1) + (K - 1) - 1;
    constexpr int B_ZY = (K - 1) * (K - 1) + (K - 2);
    const int lane = lane_id();

#pragma unroll
    for (int d = 0; d < R; ++d)
        if (lane == d) s.mark[mem[d]] = (MarkT<K>)(s.mark[mem[d]] | FLAG);
    int r0[R], pre[R + 1];
    pre[0] = 0;
#pragma unroll
    for (int d = 0; d < R; ++d) {
        r0[d] = uniform(s.urow[mem[d]]);
        pre[d + 1] = pre[d] + uniform(s.urow[mem[d] + 1]) - r0[d];
    }
    const int total = pre[R];
    __syncthreads();

    // 1. cells of adj(X)
    int ncell = 0, nadj = 0;
    for (int base = 0; base < total; base += kWave) {
        const int a = base + lane;
        bool mine = false;
        uint32_t cell = 0, vid = 0, mk = 0;
        if (a < total) {
            int d;
            const int e = member_entry<R>(pre, r0, a, &d);
            vid = s.uadj[e] >> 2;
            mk = s.mark[vid];
            mine = !is_member<K>(mk) && !(mk & lower_members<K>(d));
            cell = cell_of<K>(mk);
        }
        bool fresh = false;
        if (mine) fresh = atomicAdd(&c.cnt[cell], 1u) == 0u;
        const unsigned long long bal = __ballot(fresh);
        if (fresh) {
            const int at = ncell + (int)lanes_below(bal);
            c.list[at] = (uint8_t)cell;
            c.pos[cell] = (uint8_t)at;
        }
        if (mine) {
            // the cell's position into the mark's top bits (15 and up: none)
            const uint32_t p = c.pos[cell];
            s.mark[vid] = (MarkT<K>)((mk & ~kMemberFlag<K>) | ((p < 15u ? p : 0u) << kPosShift<K>));
        }
        ncell += __popcll(bal);
        nadj += __popcll(__ballot(mine));
    }
    __syncthreads();
    const bool agg = ncell <= kAggCells<K>;
    const uint32_t pairs_w = (uint32_t)nadj * (uint32_t)(nadj - 1) / 2u;  // sum of the weights
    if (s.hpending + pairs_w >= kPendingMax) flush_hash<K>(s);
    s.hpending += pairs_w;

    // 2. arc pairs inside adj(X): into the table, or +1 with the arcs and -1
    // without straight into the hash
    auto arc = [&](bool edge, int, int, uint32_t mu, uint32_t mv, uint32_t t) {
        if (agg) {
            if (edge) {
                uint32_t ia = (mu >> kPosShift<K>) & 15u, ib = (mv >> kPosShift<K>) & 15u;
                if (ia > ib) {
                    const uint32_t x = ia;
                    ia = ib;
                    ib = x;
                    t = ((t & 1u) << 1) | (t >> 1);
                }
                atomicAdd(&c.agg[3u * (ib * (ib + 1u) / 2u + ia) + t - 1u], 1u);
            }
        } else {
            const uint32_t cm = cx | code_bits<K>(mu & ~kMemberFlag<K>, K - 2) |
                                code_bits<K>(mv & ~kMemberFlag<K>, K - 1);
            const uint32_t ct = cm | ((t & 1u) << B_YZ) | ((t >> 1) << B_ZY);
            bool et = edge, em = edge;
            const uint32_t it = class_of<K>(s, et, ct), im = class_of<K>(s, em, cm);
            if (s.hpending >= kPendingMax - 2u * kWave) flush_hash<K>(s);
            count_codes<K>(s, et, it);
            uncount_codes<K>(s, em, im);
        }
    };
    if (nap >= 0) {
        // the parent's arc pairs, less those at z
        const int z = mem[R - 1];
        for (int ib = 0; ib < nap; ib += kWave) {
            const int i = ib + lane;
            bool edge = false;
            uint32_t mu = 0, mv = 0, t = 0;
            if (i < nap) {
                const uint32_t ent = c.ap[i];
                const int u = (int)(ent & 0x1FFFu), v = (int)((ent >> 13) & 0x1FFFu);
                t = ent >> 26;
                edge = u != z && v != z;
                mu = s.mark[u];
                mv = s.mark[v];
            }
            arc(edge, 0, 0, mu, mv, t);
        }
        // arcs at the vertices z brings (no mark bits of P): to any vertex
        // of adj(P), or to another new one above them
        const uint32_t of_p = lower_members<K>(R - 1);
        scan_taken<K, R>(
            s, c, pre, r0, R - 1,
            [of_p](int v, int u, uint32_t mv) { return (mv & of_p) != 0u || v > u; }, arc);
    } else {
        scan_taken<K, R>(s, c, pre, r0, 0, [](int v, int u, uint32_t) { return v > u; }, arc);
    }

    // 3. pairs of cells (Y <= Z): C(|Y|,2) or |Y||Z| k-sets of motif(X, Y, Z),
    // less the arc pairs of the table, which go to their own classes
    const int npairs = ncell * (ncell + 1) / 2;
    for (int pb = 0; pb < npairs; pb += kWave) {
        const int p = pb + lane;
        bool valid = false;
        uint32_t code = 0, w = 0, e1 = 0, e2 = 0, e3 = 0;
        if (p < npairs) {
            // p = z(z+1)/2 + y with y <= z
            int z = (int)((__builtin_sqrtf(8.0f * (float)p + 1.0f) - 1.0f) * 0.5f);
            if ((z + 1) * (z + 2) / 2 <= p) ++z;
            if (z * (z + 1) / 2 > p) --z;
            const int y = p - z * (z + 1) / 2;
            const uint32_t cy = c.list[y], cz = c.list[z];
            const uint32_t ny = c.cnt[cy], nz = c.cnt[cz];
            w = y == z ? ny * (ny - 1u) / 2u : ny * nz;
            if (agg) {
                uint32_t *row = c.agg + 3 * p;
                e1 = row[0];
                e2 = row[1];
                e3 = row[2];
                row[0] = row[1] = row[2] = 0u;
                w -= e1 + e2 + e3;
            }
            code = cx | code_bits<K>(mark_of_cell<K>(cy), K - 2) |
                   code_bits<K>(mark_of_cell<K>(cz), K - 1);
            valid = w > 0;
        }
        if (!(agg && __ballot(e1 | e2 | e3))) {
            hash_insert<K>(s, valid, class_of<K>(s, valid, code), w);
            continue;
        }
        // up to four (code, count) items a lane -- the pair less its arcs,
        // and its arc pairs by type -- compacted through the scratch into
        // one insert when they fit a wave
        const uint32_t nl = (valid ? 1u : 0u) + (e1 ? 1u : 0u) + (e2 ? 1u : 0u) + (e3 ? 1u : 0u);
        uint32_t incl = nl;
        incl = (uint32_t)wave_incl_sum((int)incl);
        const int items = __builtin_amdgcn_readlane((int)incl, kWave - 1);
        if (items <= kWave) {
            uint32_t *qk = s.scratch, *qn = s.scratch + kWave;
            uint32_t at = incl - nl;
            if (valid) {
                qk[at] = code;
                qn[at++] = w;
            }
            if (e1) {
                qk[at] = code | (1u << B_YZ);
                qn[at++] = e1;
            }
            if (e2) {
                qk[at] = code | (1u << B_ZY);
                qn[at++] = e2;
            }
            if (e3) {
                qk[at] = code | (1u << B_YZ) | (1u << B_ZY);
                qn[at] = e3;
            }
            __syncthreads();
            bool mine = lane < items;
            const uint32_t ic = mine ? qk[lane] : 0u, in = mine ? qn[lane] : 0u;
            __syncthreads();
            hash_insert<K>(s, mine, class_of<K>(s, mine, ic), in);
        } else {
            hash_insert<K>(s, valid, class_of<K>(s, valid, code), w);
            bool v1 = e1 > 0, v2 = e2 > 0, v3 = e3 > 0;
            const uint32_t i1 = class_of<K>(s, v1, code | (1u << B_YZ));
            const uint32_t i2 = class_of<K>(s, v2, code | (1u << B_ZY));
            const uint32_t i3 = class_of<K>(s, v3, code | (1u << B_YZ) | (1u << B_ZY));
            hash_insert<K>(s, v1, i1, e1);
            hash_insert<K>(s, v2, i2, e2);
            hash_insert<K>(s, v3, i3, e3);
        }
    }

    // reset the cell counts and the member flags
    for (int i = lane; i < ncell; i += kWave) c.cnt[c.list[i]] = 0u;
#pragma unroll
    for (int d = 0; d < R; ++d)
        if (lane == d) s.mark[mem[d]] = (MarkT<K>)(s.mark[mem[d]] & ~FLAG);
    __syncthreads();
}

// node with members s_0..s_D (D < k-3): its children jlo..jhi-1 become
// member D+1; at D+1 = k-3 each child completes a core
template <int K, int D, int V>
__device__ void visit_core(EnumState<K, V> &s, const CoreLds &c, const int (&st)[K - 1],
                           uint32_t code, int jlo, int jhi, int (&mem)[K])
{
    int rem[D + 1];
    int total = 0;
#pragma unroll
    for (int q = 0; q <= D; ++q) {
        rem[q] = s.len[q] - st[q];
        total += rem[q];
    }
    const int hi = total < jhi ? total : jhi;
    // a parent of cores (k >= 5): its arc list, shared by the children
    int nap = -1;
    if constexpr (D + 1 == K - 3) {
        if (jlo < hi && c.ap && !(s.flags & kDebugNoShare)) nap = parent_arcs<K, D + 1>(s, c, mem);
    }
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
        const uint32_t ccode =
            code | code_bits<K>((uint32_t)uniform((int)s.mark[x]) & ~kMemberFlag<K>, D + 1);
        mem[D + 1] = x;
        if constexpr (D + 1 == K - 3) {
            const Held held = push_marks_held<K, D + 1>(s, x);
            core_node<K>(s, c, mem, ccode, nap);
            core_pop<K, D + 1>(s, x, held);
        } else {
            const Held held = push_held<K, D + 1>(s, x);
            int cst[K - 1];
#pragma unroll
            for (int q = 0; q < K - 1; ++q)
                cst[q] = q < L ? s.len[q] : (q == L ? o + 1 : (q <= D ? st[q] : 0));
            visit_core<K, D + 1>(s, c, cst, ccode, 0, INT_MAX, mem);
            core_pop<K, D + 1>(s, x, held);
        }
    }
}

// A unit: k = 3, the core {v}; k = 4, the core {v, w_i}; k >= 5, the cores
// below children jlo..jhi-1 of the node (v, w_i).
template <int K, int V>
__device__ void run_core_unit(EnumState<K, V> &s, const CoreLds &c, int v, int i, uint32_t range)
{
    int mem[K];
#pragma unroll
    for (int q = 0; q < K; ++q) mem[q] = 0;
    mem[0] = v;
    s.root = v;
    if constexpr (K == 3) {
        const Held held0 = push_marks_held<K, 0>(s, v);
        core_node<K>(s, c, mem, 0u, -1);
        core_pop<K, 0>(s, v, held0);
    } else {
        const Held held0 = push_held<K, 0>(s, v);
        if (i < s.len[0]) {
            const int x = uniform((int)s.seg[i]);
            const uint32_t code = code_bits<K>((uint32_t)uniform((int)s.mark[x]) & ~kMemberFlag<K>, 1);
            mem[1] = x;
            if constexpr (K == 4) {
                const Held held1 = push_marks_held<K, 1>(s, x);
                core_node<K>(s, c, mem, code, -1);
                core_pop<K, 1>(s, x, held1);
            } else {
                const Held held1 = push_held<K, 1>(s, x);
                int st[K - 1];
#pragma unroll
                for (int q = 0; q < K - 1; ++q) st[q] = 0;
                st[0] = i + 1;
                const bool full = range == kFullChild;
                visit_core<K, 1>(s, c, st, code, full ? 0 : (int)(range & 0xFFFFu),
                                 full ? INT_MAX : (int)(range >> 16), mem);
                core_pop<K, 1>(s, x, held1);
            }
        } else if (lane_id() == 0) {
            atomicAdd(s.errors, 1u);
        }
        core_pop<K, 0>(s, v, held0);
    }
}

template <int K, int V>
__device__ __forceinline__ void core_body(const DevGraph *graphs, const int4 *units,
                                          uint32_t unit_cap, uint32_t unit_end, uint32_t *counters,
                                          const uint32_t *table, uint32_t num_classes,
                                          unsigned long long *hist_base, const EnumConfig &cfg)
{
    extern __shared__ uint32_t lds[];
    EnumState<K, V> s;
    const LdsLayout lay = lds_layout(K, cfg.max_n, cfg.seg_cap, cfg.hash_bits, false, kCoreSegs<K>);
    char *base = reinterpret_cast<char *>(lds);
    CoreLds c;
    c.cnt = reinterpret_cast<uint32_t *>(base + lay.total);
    c.list = reinterpret_cast<uint8_t *>(c.cnt + kCells<K>);
    c.pos = c.list + ((kCells<K> + 3) & ~3);
    uint32_t *after_pos = reinterpret_cast<uint32_t *>(c.pos + ((kCells<K> + 3) & ~3));
    c.uid = kPackedUid<K> ? nullptr : after_pos;
    c.agg = kPackedUid<K> ? after_pos : after_pos + kWave;
    c.ap = cfg.wave_scratch ? cfg.wave_scratch + (size_t)blockIdx.x * kParentArcCap : nullptr;
    for (int i = lane_id(); i < kCells<K>; i += kWave) c.cnt[i] = 0u;
    for (int i = lane_id(); i < kAggWords<K>; i += kWave) c.agg[i] = 0u;
    init_state<K>(s, base, lay, cfg, counters, table, num_classes);
    s.class_keys = true;
    // flushed at three quarters full, and not at the end of a unit: class
    // ids spread evenly, so few inserts probe far, and each flush then
    // carries more of the counts (the graph's next units add to the same
    // classes)
    s.hlimit = (int)((s.hmask >> 1) + (s.hmask >> 2));
    s.hunit = INT_MAX;
    // heavy units first at k = 5 only (k = 3 and 6 measured slower with it)
    for_each_unit<K == 5, K>(s, graphs, units, unit_cap, unit_end, counters, hist_base, cfg,
                     [&](int v, int i, uint32_t range) { run_core_unit<K>(s, c, v, i, range); });
}

template <int K>
__global__ __launch_bounds__(kWave) void core_kernel(const DevGraph *graphs, const int4 *units,
                                                     uint32_t unit_cap, uint32_t unit_end,
                                                     uint32_t *counters,
                                                     const uint32_t *table, uint32_t num_classes,
                                                     unsigned long long *hist_base,
                                                     EnumConfig cfg)
{
    core_body<K, 0>(graphs, units, unit_cap, unit_end, counters, table, num_classes, hist_base, cfg);
}

// the build that honours the test hooks of the hash
template <int K>
__global__ __launch_bounds__(kWave) void core_debug_kernel(const DevGraph *graphs, const int4 *units,
                                                           uint32_t unit_cap, uint32_t unit_end,
                                                           uint32_t *counters,
                                                           const uint32_t *table, uint32_t num_classes,
                                                           unsigned long long *hist_base,
                                                           EnumConfig cfg)
{
    core_body<K, kVarDebug>(graphs, units, unit_cap, unit_end, counters, table, num_classes,
                            hist_base, cfg);
}

// hist[g][c] := raw / core_mult[c]; a raw count that is not a multiple (or
// is negative as a 64-bit integer) is a device-side error.
__global__ void core_divide_kernel(unsigned long long *hist, uint32_t num_classes,
                                   const uint8_t *mult, uint32_t *errors)
{
    unsigned long long *h = hist + (size_t)blockIdx.y * num_classes;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < num_classes;
         i += gridDim.x * blockDim.x) {
        const unsigned long long raw = h[i];
        if (raw == 0) continue;
        const uint32_t m = mult[i];
        if (m == 0 || (long long)raw < 0) {
            atomicAdd(errors, 1u);
            continue;
        }
        const unsigned long long q = raw / m;
        if (q * m != raw) atomicAdd(errors, 1u);
        h[i] = q;
    }
}

// Per-wave hash slots of the core kernel (keys are class ids).  Its LDS
// sets how many waves a CU holds, and the kernel's speed follows that
// count, so the hash trades capacity for waves: on the k = 5 batch 256
// slots flushed at three quarters (7.5 KB of LDS a wave) take 21.2 ms, 512
// slots 23.9 ms and 128 slots 28.2 ms at three quarters; flushed at half,
// 256 slots took 27.5 ms.
#ifndef MK_CORE_HASH_BITS_K5
#define MK_CORE_HASH_BITS_K5 8
#endif
int core_hash_bits(int k) { return k == 5 ? MK_CORE_HASH_BITS_K5 : kHashBits; }

int core_lds_bytes(int k, int max_n, int seg_cap)
{
    return lds_layout(k, max_n, seg_cap, core_hash_bits(k), false, k - 3).total + core_extra_bytes(k);
}

template <int K>
static const void *core_fn(bool debug)
{
    return debug ? reinterpret_cast<const void *>(&core_debug_kernel<K>)
                 : reinterpret_cast<const void *>(&core_kernel<K>);
}

int core_max_blocks_per_cu(int k, int lds_bytes, int *blocks)
{
    const void *fn = nullptr;
    switch (k) {
    case 3: fn = core_fn<3>(false); break;
    case 4: fn = core_fn<4>(false); break;
    case 5: fn = core_fn<5>(false); break;
    case 6: fn = core_fn<6>(false); break;
    default: return fail(MK_ERANGE, "k=%d outside 3..6", k);
    }
    MK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, fn, kWave, (size_t)lds_bytes));
    return MK_OK;
}

int launch_core(int k, const DevGraph *d_graphs, const int4 *units, uint32_t unit_cap,
                uint32_t unit_end, uint32_t *counters, const uint32_t *table, uint32_t num_classes,
                unsigned long long *hist_base, const EnumConfig &cfg, int grid, int lds_bytes,
                hipStream_t stream)
{
    if (grid <= 0) return MK_OK;
    const bool debug = (cfg.variant & kVarDebug) != 0;
    const void *fn = nullptr;
    switch (k) {
    case 3: fn = core_fn<3>(debug); break;
    case 4: fn = core_fn<4>(debug); break;
    case 5: fn = core_fn<5>(debug); break;
    case 6: fn = core_fn<6>(debug); break;
    default: return fail(MK_ERANGE, "k=%d outside 3..6", k);
    }
    EnumConfig c = cfg;
    void *args[] = {(void *)&d_graphs, (void *)&units, (void *)&unit_cap, (void *)&unit_end,
                    (void *)&counters, (void *)&table, (void *)&num_classes, (void *)&hist_base,
                    (void *)&c};
    MK_HIP(hipLaunchKernel(fn, dim3(grid), dim3(kWave), args, (size_t)lds_bytes, stream));
    MK_HIP(hipGetLastError());
    return MK_OK;
}

int launch_core_divide(unsigned long long *hist, int ng, uint32_t num_classes,
                       const uint8_t *mult, uint32_t *counters, hipStream_t stream)
{
    if (ng <= 0 || num_classes == 0) return MK_OK;
    constexpr int kThreads = 256;
    const uint32_t blocks = std::min<uint32_t>((num_classes + kThreads * 4 - 1) / (kThreads * 4), 4096u);
    hipLaunchKernelGGL(core_divide_kernel, dim3(blocks, (unsigned)ng), dim3(kThreads), 0, stream,
                       hist, num_classes, mult, &counters[kErrors]);
    MK_HIP(hipGetLastError());
    return MK_OK;
}

}  // namespace mk
