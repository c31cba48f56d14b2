// Wave-level building blocks of the ESU walk shared by the enumeration
// kernel (every k-set, Section 3.2's O(1) lookup per subgraph) and the
// (k-2)-set counting kernel (Section 3's loop over L_{k-2}): per-wave LDS
// marks and extension segments, member push/pop, the per-wave hash of
// pending (code, count) pairs with its flush into the histogram, and the
// persistent work-queue loop.
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
// Counts are added to a small per-wave LDS hash of pending (code, count)
// pairs; only its flush looks codes up in the code -> class table and adds
// to the graph's histogram with 64-bit atomics.
#pragma once

#include <climits>
#include <type_traits>

#include "internal.h"

namespace mk {



// members whose extension segment is kept: positions 0..k-3 (k >= 4; the
// last two levels are flat), positions 0..1 for k = 3
template <int K>
constexpr int kSegments = K == 3 ? 2 : K - 2;
constexpr int kScratchWords = 3 * kWave;
// Compile-time tuning knobs (build flags may override them).
#ifndef MK_HASH_BITS
#define MK_HASH_BITS 8   // log2 of the per-wave hash slots
#endif
#ifndef MK_HEAVY_GRAB
#define MK_HEAVY_GRAB 4  // units per grab of the first sweep, in grabs of the second
#endif
#ifndef MK_MERGE_ROUNDS
#define MK_MERGE_ROUNDS 1  // ballot rounds merging equal codes before the hash
#endif
#ifndef MK_ROW_MIN
#define MK_ROW_MIN 32    // see kRowMin
#endif

// Per-wave hash of pending (code, count) pairs; flushed to the histogram when
// half full (the core kernel: three quarters), at the end of a unit once a
// quarter full (not in the core kernel), on a graph switch and at exit.
constexpr int kHashBits = MK_HASH_BITS;  // the enumeration kernel's; see EnumConfig
constexpr int kHashProbes = 8;
constexpr uint32_t kEmpty = 0xFFFFFFFFu;
// A flush is forced once this many subgraphs are pending, so no 32-bit slot
// count can overflow (every insert adds less than 2^31 on top).
constexpr uint32_t kPendingMax = 1u << 30;
// Rows of the last-level pair triangle, and children's lists, at least this
// long are processed one at a time with their first vertex wave-uniform.
constexpr int kRowMin = MK_ROW_MIN;

// extension segment entries: u16 vertex ids, u32 with global marks
template <int V>
using SegT = typename std::conditional<(V & kVarGlobal) != 0, uint32_t, uint16_t>::type;

// Byte offsets of one wave's LDS: marks (n x 2 or 4 bytes; none when they
// are in global memory), extension segments (u16, or u32 with global
// marks), scratch, hash keys and counts; each part 4-byte aligned.
struct LdsLayout {
    int seg, scratch, total;
};

__host__ __device__ inline LdsLayout lds_layout(int k, int max_n, int seg_cap, int hash_bits,
                                                bool global_marks = false, int segs = -1)
{
    if (segs < 0) segs = k == 3 ? 2 : k - 2;
    const int mark_bytes = global_marks ? 0 : (((k <= 5 ? 2 : 4) * max_n + 3) & ~3);
    const int seg_bytes = ((global_marks ? 4 : 2) * segs * seg_cap + 3) & ~3;
    LdsLayout l;
    l.seg = mark_bytes;
    l.scratch = l.seg + seg_bytes;
    l.total = l.scratch + 4 * (kScratchWords + 2 * (1 << hash_bits));
    return l;
}

// Marks hold, for members at positions 0..kSegments-1, the "in" bits spread
// at stride k-1 (highest at (kSegments-1)(k-1)) and then one "out" bit per
// position: 5 / 6 / 12 / 20 bits for k = 3 / 4 / 5 / 6, so 16-bit marks do
// for k <= 5 in LDS.  Marks in device memory are 32-bit for every k (room
// for the extension-list tags of last_two_cells).
template <int K, int V = 0>
using MarkT = typename std::conditional<K <= 5 && (V & kVarGlobal) == 0, uint16_t, uint32_t>::type;

template <int K, int V = 0>
struct EnumState {
    static constexpr int OUTB = (kSegments<K> - 1) * (K - 1) + 1;
    static constexpr uint32_t INMASK = (1u << OUTB) - 1u;
    static_assert(OUTB + kSegments<K> <= 8 * (int)sizeof(MarkT<K, V>), "mark bits do not fit");
    MarkT<K, V> *mark;          // LDS, or this wave's global array (kVarGlobal)
    SegT<V> *seg;               // vertex ids
    int seg_cap;
    int root;
    GPtr<const int32_t> urow;
    GPtr<const uint32_t> uadj;
    GPtr<const uint32_t> bits_out;  // row w bit u: arc w -> u
    GPtr<const uint32_t> bits_in;   // row w bit u: arc u -> w
    int words;
    uint32_t *scratch;          // 3 x 64 words of LDS per wave
    uint32_t *hkey;             // per-wave LDS hash: code (kEmpty = free)
    uint32_t *hcnt;             //   and its pending count
    int hshift;                 // 32 - log2(hash slots)
    uint32_t hmask;             // hash slots - 1
    int hused;                  // keys in the hash (wave-uniform)
    int hlimit;                 // flush once hused exceeds this
    int hunit;                  //   or, after a unit, exceeds this
    uint32_t hpending;          // subgraphs pending in the hash (wave-uniform)
    bool class_keys;            // hash keys are class ids, not codes
    uint32_t flags;             // kDebug* bits
    unsigned long long *hist;
    const uint32_t *table;
    uint32_t num_classes;
    uint32_t *errors;
    int len[K - 1];
};

__device__ __forceinline__ int lane_id() { return (int)threadIdx.x; }

__device__ __forceinline__ int uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }

// Inclusive prefix sum across the wave by DPP moves (rows of 16 lanes
// shifted by 1, 2, 4 and 8, then each row's last lane broadcast into the
// next rows): six VALU operations, where the lane-shuffle loop waits on six
// dependent LDS-crossbar permutes.  Every lane must be active.
__device__ __forceinline__ int wave_incl_sum(int x)
{
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xF, 0xF, false);  // row_shr:1
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xF, 0xF, false);  // row_shr:2
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xF, 0xF, false);  // row_shr:4
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xF, 0xF, false);  // row_shr:8
    x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xA, 0xF, false);  // row_bcast:15
    x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xC, 0xF, false);  // row_bcast:31
    return x;
}

// Inclusive prefix maximum across the wave (the same DPP pattern; values
// must be >= 0).
__device__ __forceinline__ int wave_incl_max(int x)
{
    x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x111, 0xF, 0xF, false));
    x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x112, 0xF, 0xF, false));
    x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x114, 0xF, 0xF, false));
    x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x118, 0xF, 0xF, false));
    x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x142, 0xA, 0xF, false));
    x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x143, 0xC, 0xF, false));
    return x;
}

// Flat scan over the lists of the wave's lanes: lane j owns the entries
// [incl_j - deg_j, incl_j) (incl the inclusive prefix of the degrees).  The
// source lane of entry fb + lane: every lane whose range meets [fb, fb + 64)
// writes its id at its first entry there into buf (64 words of LDS), and a
// prefix maximum carries each id over the entries after it -- in place of a
// six-step binary search of dependent LDS reads per entry.  Every lane must
// be active.
__device__ __forceinline__ int flat_source(uint32_t *buf, int incl, int deg, int fb)
{
    const int lane = (int)threadIdx.x;
    const int excl = incl - deg;
    buf[lane] = 0u;
    __syncthreads();
    if (deg > 0 && excl < fb + kWave && incl > fb) buf[excl > fb ? excl - fb : 0] = (uint32_t)lane;
    __syncthreads();
    return wave_incl_max((int)buf[lane]);
}

__device__ __forceinline__ uint32_t lanes_below(unsigned long long mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// both mark bits of member position d for a neighbour of type t
template <int K>
__device__ __forceinline__ uint32_t mark_bits(int d, uint32_t t)
{
    return ((t & 1u) << (d * (K - 1))) | (((t >> 1) & 1u) << (EnumState<K>::OUTB + d));
}

// code bits contributed by a vertex with mark m joining at position p >= 1
template <int K>
__device__ __forceinline__ uint32_t code_bits(uint32_t m, int p)
{
    return ((m >> EnumState<K>::OUTB) << (p * (K - 1))) | ((m & EnumState<K>::INMASK) << (p - 1));
}

// s_D := x.  Builds seg[D] (new exclusive extension vertices, ascending) and
// ORs position D's bits into the marks of x's neighbours.
template <int K, int D, int V>
__device__ __forceinline__ void push(EnumState<K, V> &s, int x)
{
    const int lane = lane_id();
    const int r0 = uniform(s.urow[x]);
    const int r1 = uniform(s.urow[x + 1]);
    SegT<V> *seg = s.seg + D * s.seg_cap;
    int cnt = 0;
    for (int base = r0; base < r1; base += kWave) {
        const int e = base + lane;
        const bool valid = e < r1;
        const uint32_t ent = valid ? s.uadj[e] : 0u;
        const int y = (int)(ent >> 2);
        const uint32_t m = valid ? s.mark[y] : 1u;
        const bool fresh = valid && y > s.root && m == 0u;
        const unsigned long long bal = __ballot(fresh);
        if (fresh) seg[cnt + (int)lanes_below(bal)] = (SegT<V>)y;
        cnt += __popcll(bal);
        if (valid) s.mark[y] = (MarkT<K, V>)(m | mark_bits<K>(D, ent & 3u));
    }
    s.len[D] = cnt;
    __syncthreads();
}

// undo push<D>(x)
template <int K, int D, int V>
__device__ __forceinline__ void pop(EnumState<K, V> &s, int x)
{
    const int lane = lane_id();
    const int r0 = uniform(s.urow[x]);
    const int r1 = uniform(s.urow[x + 1]);
    const uint32_t keep = ~mark_bits<K>(D, 3u);
    for (int base = r0; base < r1; base += kWave) {
        const int e = base + lane;
        if (e < r1) {
            const int y = (int)(s.uadj[e] >> 2);
            s.mark[y] = (MarkT<K, V>)(s.mark[y] & keep);
        }
    }
    __syncthreads();
}

// A member's list when it fits one wave: each lane keeps its entry and the
// neighbour's mark from before the push, so the pop restores the marks
// without reading the list again (deeper levels undo their own bits, so the
// marks at the pop are exactly these plus the member's).
struct Held {
    uint32_t ent;  // this lane's list entry (lanes < n)
    uint32_t m;    // the neighbour's mark before the push
    int n;         // list length (wave-uniform)
};

// push<D>(x), keeping the list for pop_held
template <int K, int D, int V>
__device__ __forceinline__ Held push_held(EnumState<K, V> &s, int x)
{
    const int lane = lane_id();
    const int r0 = uniform(s.urow[x]);
    const int r1 = uniform(s.urow[x + 1]);
    Held h;
    h.n = r1 - r0;
    h.ent = 0u;
    h.m = 0u;
    if (h.n > kWave) {
        push<K, D>(s, x);
        return h;
    }
    SegT<V> *seg = s.seg + D * s.seg_cap;
    const bool valid = lane < h.n;
    if (valid) h.ent = s.uadj[r0 + lane];
    const int y = (int)(h.ent >> 2);
    if (valid) h.m = s.mark[y];
    const bool fresh = valid && y > s.root && h.m == 0u;
    const unsigned long long bal = __ballot(fresh);
    if (fresh) seg[(int)lanes_below(bal)] = (SegT<V>)y;
    if (valid) s.mark[y] = (MarkT<K, V>)(h.m | mark_bits<K>(D, h.ent & 3u));
    s.len[D] = __popcll(bal);
    __syncthreads();
    return h;
}

// undo push_held<D>(x)
template <int K, int D, int V>
__device__ __forceinline__ void pop_held(EnumState<K, V> &s, int x, const Held &h)
{
    if (h.n > kWave) {
        pop<K, D>(s, x);
        return;
    }
    if (lane_id() < h.n) s.mark[h.ent >> 2] = (MarkT<K, V>)h.m;
    __syncthreads();
}

// add n to the histogram bin of code (table lookup + global 64-bit atomic)
template <int K, int V>
__device__ __forceinline__ void add_global(EnumState<K, V> &s, uint32_t code, uint32_t n)
{
    const uint32_t id = s.class_keys ? code : s.table[code];
    // n is a 32-bit two's complement count (negative only in the (k-2)-set
    // counting); sign-extended, the 64-bit sums stay exact modulo 2^64
    if (id < s.num_classes) atomicAdd(&s.hist[id], (unsigned long long)(long long)(int32_t)n);
    else atomicAdd(s.errors, 1u);
}

// move the wave's pending counts to the histogram and empty the hash
template <int K, int V>
__device__ __forceinline__ void flush_hash(EnumState<K, V> &s)
{
    __syncthreads();
    for (int i = lane_id(); i <= (int)s.hmask; i += kWave) {
        const uint32_t key = s.hkey[i];
        if (key != kEmpty) {
            if (s.hcnt[i] != 0u) add_global<K>(s, key, s.hcnt[i]);
            s.hkey[i] = kEmpty;
            s.hcnt[i] = 0u;
        }
    }
    s.hused = 0;
    s.hpending = 0;
    __syncthreads();
}

// Add n to the pending count of code for every lane with `mine` set: the
// wave's LDS hash (linear probing); a lane that finds no slot within
// kHashProbes goes straight to the histogram.  Flushes when half full.
template <int K, int V>
__device__ __forceinline__ void hash_insert(EnumState<K, V> &s, bool mine, uint32_t code, uint32_t n)
{
    bool fresh = false;
    if constexpr ((V & kVarDebug) != 0) {
        if (s.flags & kDebugNoHash) {
            if (mine) add_global<K>(s, code, n);
            return;
        }
    }
    if (mine) {
        // one compare-and-swap either claims an empty slot or finds the code
        // already there; only a collision probes on
        uint32_t h = (code * 2654435761u) >> s.hshift;
        uint32_t old = atomicCAS(&s.hkey[h], kEmpty, code);
        bool ok = old == kEmpty || old == code;
        for (int p = 1; p < kHashProbes && !ok; ++p) {
            h = (h + 1) & s.hmask;
            old = atomicCAS(&s.hkey[h], kEmpty, code);
            ok = old == kEmpty || old == code;
        }
        if (ok) {
            fresh = old == kEmpty;
            atomicAdd(&s.hcnt[h], n);
        } else {
            add_global<K>(s, code, n);
        }
    }
    s.hused += __popcll(__ballot(fresh));
    if (s.hused > s.hlimit || s.hpending >= kPendingMax ||
        ((V & kVarDebug) != 0 && (s.flags & kDebugFlushAlways)))
        flush_hash<K>(s);
}

// count one code per valid lane.  MK_MERGE_ROUNDS ballot rounds merge the
// lanes that share the first remaining lane's code; every code left goes
// into the hash.
template <int K, int V>
__device__ __forceinline__ void count_codes(EnumState<K, V> &s, bool valid, uint32_t code)
{
    const int lane = lane_id();
    unsigned long long act = __ballot(valid);
    if (!act) return;
    s.hpending += (uint32_t)__popcll(act);
    uint32_t n = 1;
#pragma unroll
    for (int r = 0; r < MK_MERGE_ROUNDS; ++r) {
        if (!act) break;
        const int l = __builtin_ctzll(act);
        const uint32_t c0 = (uint32_t)__builtin_amdgcn_readlane((int)code, l);
        const unsigned long long eq = __ballot(code == c0) & act;
        if (lane == l) n = (uint32_t)__popcll(eq);
        else if ((eq >> lane) & 1ull) n = 0;
        act &= ~eq;
    }
    hash_insert<K>(s, valid && n > 0, code, n);
}


// count codes with weight -1 (merged like count_codes)
template <int K, int V>
__device__ __forceinline__ void uncount_codes(EnumState<K, V> &s, bool valid, uint32_t code)
{
    const int lane = lane_id();
    unsigned long long act = __ballot(valid);
    if (!act) return;
    s.hpending += (uint32_t)__popcll(act);
    uint32_t n = 1;
    const int l = __builtin_ctzll(act);
    const uint32_t c0 = (uint32_t)__builtin_amdgcn_readlane((int)code, l);
    const unsigned long long eq = __ballot(code == c0) & act;
    if (lane == l) n = (uint32_t)__popcll(eq);
    else if ((eq >> lane) & 1ull) n = 0;
    hash_insert<K>(s, valid && n > 0, code, 0u - n);
}

// Set up a wave's state on its LDS (marks zero, hash empty).
template <int K, int V>
__device__ __forceinline__ void init_state(EnumState<K, V> &s, char *base, const LdsLayout &lay,
                                           const EnumConfig &cfg, uint32_t *counters,
                                           const uint32_t *table, uint32_t num_classes)
{
    if constexpr ((V & kVarGlobal) != 0)
        s.mark = reinterpret_cast<MarkT<K, V> *>(cfg.marks) + (size_t)blockIdx.x * cfg.mark_stride;
    else
        s.mark = reinterpret_cast<MarkT<K, V> *>(base);
    s.seg = reinterpret_cast<SegT<V> *>(base + lay.seg);
    s.seg_cap = cfg.seg_cap;
    s.flags = cfg.flags;
    s.scratch = reinterpret_cast<uint32_t *>(base + lay.scratch);
    s.hkey = s.scratch + kScratchWords;
    s.hshift = 32 - cfg.hash_bits;
    s.hmask = (1u << cfg.hash_bits) - 1u;
    s.hcnt = s.hkey + s.hmask + 1;
    s.hused = 0;
    s.hlimit = (int)(s.hmask >> 1);
    s.hunit = (int)((s.hmask + 1) >> 2);
    s.hpending = 0;
    s.class_keys = false;
    for (int i = lane_id(); i <= (int)s.hmask; i += kWave) {
        s.hkey[i] = kEmpty;
        s.hcnt[i] = 0u;
    }
    s.bits_out = nullptr;
    s.bits_in = nullptr;
    s.words = 0;
    s.table = table;
    s.num_classes = num_classes;
    s.errors = &counters[kErrors];
    s.root = 0;
    s.urow = nullptr;
    s.uadj = nullptr;
    s.hist = nullptr;
    // global marks are zeroed when allocated and every pop restores them
    if constexpr ((V & kVarGlobal) == 0)
        for (int i = lane_id(); i < cfg.max_n; i += kWave) s.mark[i] = 0;
    __syncthreads();
}

// The persistent loop: take units from the kQueues queues (own XCD's range
// first) and call run(v, i, range) for each.  When the unit's graph changes,
// on_switch(gi) runs first (a kernel flushes what it holds for the previous
// graph there) and the state is pointed at the new graph; after_unit() runs
// after every unit.  With HeavyFirst the ranges are swept twice: first for
// the units the planner marked heavy (grabs of MK_HEAVY_GRAB times the
// usual units, their marks read by the lanes at once), then for the rest,
// so that the costliest estimates start early and the launch ends on short
// units.  That takes the k = 5 core kernel from 18.55 to 17.53 ms on its
// benchmark batch; the k = 6 enumeration kernel lost 1-15% with it (over
// shifts 0-2 and grabs 2-4), the core kernel 39% at k = 3 and 88% at
// k = 6, and those sweep once.
template <bool HeavyFirst, int K, int V, typename Run, typename Switch, typename After>
__device__ __forceinline__ void unit_loop(EnumState<K, V> &s, const DevGraph *graphs,
                                          const int4 *units, uint32_t unit_cap, uint32_t unit_end,
                                          uint32_t *counters, const EnumConfig &cfg, Run run,
                                          Switch on_switch, After after_unit)
{
    const uint32_t navail = counters[kNumUnits];
    const uint32_t cap = unit_cap < unit_end ? unit_cap : unit_end;
    const uint32_t end = navail < cap ? navail : cap;
    const uint32_t begin = counters[kSliceBegin];
    const uint32_t span = end > begin ? end - begin : 0u;
    // units per grab: about 1/32 of a wave's share, 1..16
    uint32_t chunk = cfg.chunk ? cfg.chunk : span / (gridDim.x * 32u);
    chunk = chunk < 1u ? 1u : (chunk > 256u ? 256u : chunk);
    if (!cfg.chunk && chunk > 16u) chunk = 16u;
    // two sweeps only with at least 32 units per wave (a launch of one
    // graph's units would leave most waves idle behind a few heavy grabs);
    // the first sweep's grabs: MK_HEAVY_GRAB times as many units, at most 64
    const bool two = HeavyFirst && span >= gridDim.x * 32u;
    const uint32_t chunk0 = chunk * MK_HEAVY_GRAB < (uint32_t)kWave ? chunk * MK_HEAVY_GRAB : (uint32_t)kWave;
    int cur = -1;
    auto take = [&](const int4 &u) {
        const int gi = uniform((int)((uint32_t)u.x & ~kHeavyBit));
        if (gi != cur) {
            on_switch(gi);
            s.urow = (GPtr<const int32_t>)graphs[gi].urow;
            s.uadj = (GPtr<const uint32_t>)graphs[gi].uadj;
            s.bits_out = (GPtr<const uint32_t>)graphs[gi].bits_out;
            s.bits_in = (GPtr<const uint32_t>)graphs[gi].bits_in;
            s.words = graphs[gi].words;
            cur = gi;
        }
        run(uniform(u.y), uniform(u.z), (uint32_t)uniform(u.w));
        after_unit();
    };
    const int home = (int)(blockIdx.x % kQueues);
    for (int sweep = two ? 0 : 1; sweep < 2; ++sweep) {
        const uint32_t ch = sweep == 0 ? chunk0 : chunk;
        for (int q = 0; q < kQueues; ++q) {
            const int x = (home + q) % kQueues;
            const uint32_t lo = begin + (uint32_t)((uint64_t)span * x / kQueues);
            const uint32_t hi = begin + (uint32_t)((uint64_t)span * (x + 1) / kQueues);
            uint32_t *head = &counters[(sweep == 0 ? kHeavyHeads : kQueueHeads) + x * kHeadStride];
            for (;;) {
                uint32_t idx = 0;
                if (lane_id() == 0) idx = atomicAdd(head, ch);
                idx = lo + (uint32_t)uniform((int)idx);
                if (idx >= hi) break;
                const uint32_t stop = idx + ch < hi ? idx + ch : hi;
                if (sweep == 0) {
                    const uint32_t my = idx + (uint32_t)lane_id();
                    const bool heavy =
                        my < stop && (((uint32_t)units[my].x & kHeavyBit) != 0u);
                    unsigned long long m = __ballot(heavy);
                    while (m) {
                        const int l = __builtin_ctzll(m);
                        m &= m - 1;
                        take(units[idx + (uint32_t)l]);
                    }
                } else {
                    for (; idx < stop; ++idx) {
                        const int4 u = units[idx];
                        if (two && ((uint32_t)u.x & kHeavyBit)) continue;
                        take(u);
                    }
                }
            }
        }
    }
}

// unit_loop for the kernels that count into dense histograms through the
// state's hash: flushed on a graph switch, once a quarter full after a
// unit, and at the end
template <bool HeavyFirst, int K, int V, typename Run>
__device__ __forceinline__ void for_each_unit(EnumState<K, V> &s, const DevGraph *graphs,
                                              const int4 *units, uint32_t unit_cap,
                                              uint32_t unit_end, uint32_t *counters,
                                              unsigned long long *hist_base, const EnumConfig &cfg,
                                              Run run)
{
    unit_loop<HeavyFirst>(
        s, graphs, units, unit_cap, unit_end, counters, cfg, run,
        [&](int gi) {
            if (s.hused) flush_hash<K>(s);
            s.hist = hist_base + (size_t)gi * s.num_classes;
        },
        [&] {
            if (s.hused > s.hunit) flush_hash<K>(s);
        });
    if (s.hused) flush_hash<K>(s);
}

}  // namespace mk
