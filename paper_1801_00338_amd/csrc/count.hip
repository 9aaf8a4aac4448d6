// Exact and local butterfly counts (ExactBFC, vBFC, eBFC; Sec. 4 of the
// paper) on gfx950.
//
// Work decomposition.  The start side A is chosen by the paper's rule (the
// side whose opposite has the smaller sum of squared degrees is walked as
// midpoints).  For a start u (a rank on side A) every midpoint v in N(u)
// contributes the suffix of adj_B[v] that lies above u; because adjacency
// lists are sorted by rank, that suffix begins right after u's own position
// in adj_B[v] (xpos) and no search is needed.
//
// Counting table.  C_u[w] lives in LDS as a dense window of the rank space.
// Each wedge adds one with a returning LDS atomic and the old value is what
// the pair {u, w} gains (C(c+1,2) - C(c,2) = c), so the fold C(C_u[w], 2)
// happens during the walk.
//
// Narrow starts (d_u <= 255).  C_u[w] <= d_u fits a byte.  One wavefront owns
// one start and a private 16 KiB table = a window of 2^14 ranks, so nothing
// is shared between waves and a window needs no workgroup barrier.  Every
// adjacency list of B is cut into segments at window boundaries (planning
// pass); the wave walks its midpoints' suffixes window by window in
// increasing order, skipping windows no suffix touches: in a window each
// midpoint contributes at most one contiguous sub-run.  Sub-runs are cut into
// pieces of 16 entries (4 aligned 16-byte groups), the pieces of all
// midpoints are spread over the 64 lanes (a wave prefix sum plus an LDS
// binary search map a piece to its midpoint) and each lane does four 16-byte
// loads per piece.
//
// Wide starts (d_u > 255, few).  A 512-lane workgroup shares a 64 KiB table of
// 32-bit counters (2^14 ranks); each wave walks its own chunks of 64
// midpoints in the same 16-entry pieces.
//
// Scheduling.  Starts are bucketed by their wedge count (log2) and handed out
// largest first through an atomic queue per class to persistent grids.
#include <mutex>

#include "common.h"

namespace bfc {

constexpr uint32_t INF = 0xFFFFFFFFu;
constexpr int NBUCKET = 66;
constexpr int G_SHIFT = 14;             // window = 2^14 ranks (segment granularity)
constexpr uint32_t NARROW_MAX = 255;    // byte counters: C_u[w] <= d_u <= 255 (largest threshold)

// narrow kernels: one wave per workgroup
constexpr int WT = 64;
constexpr int WTBL_BYTES = 1 << G_SHIFT;
constexpr uint32_t WTBL_WORDS = WTBL_BYTES / 4;
constexpr int WSLOTS = 4;               // midpoints per lane (4 * 64 > NARROW_MAX)
constexpr int WCHUNK = 4;               // default starts taken from the queue at once

// wide kernels: 512-lane workgroups
constexpr int NT = 512;
constexpr int TBL_WORDS = 1 << G_SHIFT; // 32-bit counters, 64 KiB

struct Plan {
    int start_r;                        // 0: starts in L, 1: starts in R
    uint32_t nA, nB;
    uint64_t m;
    const uint32_t *offA, *adjA, *xA, *offB, *adjB;
    uint32_t max_deg_A;
    uint64_t wedges;
    uint64_t split;                     // local counts: wedges per part of a wide start (0: none)
};

static int make_plan(const bfc_graph *g, int side, Plan *p) {
    if (!g) return BFC_E_NULL;
    int r;
    if (side == BFC_SIDE_AUTO) r = g->sumsq_l < g->sumsq_r;
    else if (side == BFC_SIDE_L) r = 0;
    else if (side == BFC_SIDE_R) r = 1;
    else return BFC_E_ARG;
    p->start_r = r;
    p->split = 0;
    p->m = g->n_edges;
    if (!r) {
        p->nA = g->n_left; p->nB = g->n_right;
        p->offA = g->off_l; p->adjA = g->adj_l; p->xA = g->xpos_l;
        p->offB = g->off_r; p->adjB = g->adj_r;
        p->max_deg_A = g->max_deg_l; p->wedges = g->wedges_mid_r;
    } else {
        p->nA = g->n_right; p->nB = g->n_left;
        p->offA = g->off_r; p->adjA = g->adj_r; p->xA = g->xpos_r;
        p->offB = g->off_l; p->adjB = g->adj_l;
        p->max_deg_A = g->max_deg_r; p->wedges = g->wedges_mid_l;
    }
    return BFC_OK;
}

// ------------------------------------------------------------------ planning kernels
// flag[p] = 1 where a segment starts: a row start, or a window change.
__global__ void k_seg_flags(const uint32_t *adjB, uint64_t m, uint32_t *flag) {
    for (uint64_t p = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; p < m;
         p += (uint64_t)gridDim.x * blockDim.x)
        flag[p] = (p > 0 && (adjB[p] >> G_SHIFT) != (adjB[p - 1] >> G_SHIFT)) ? 1u : 0u;
}

__global__ void k_seg_rowstarts(const uint32_t *offB, uint32_t nB, uint32_t *flag) {
    for (uint64_t v = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; v < nB;
         v += (uint64_t)gridDim.x * blockDim.x)
        if (offB[v] < offB[v + 1]) flag[offB[v]] = 1u;
}

// seg1[p] = 1 + index of the segment holding position p (inclusive scan).
__global__ void k_seg_fill(const uint32_t *adjB, uint64_t m, const uint32_t *seg1,
                           uint32_t *seg_start, uint32_t *seg_win) {
    for (uint64_t p = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; p < m;
         p += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t s = seg1[p];
        uint32_t prev = p > 0 ? seg1[p - 1] : 0;
        if (s != prev) {
            seg_start[s - 1] = (uint32_t)p;
            seg_win[s - 1] = adjB[p] >> G_SHIFT;
        }
        if (p == m - 1) seg_start[s] = (uint32_t)m;
    }
}

// Classes of starts, each with a largest-first queue: 0 dense narrow
// windows, 1 dense wide windows, 2 and 3 hash tables (few wedges, one wave /
// one workgroup per start).
constexpr int NCLASS = 4;
constexpr uint32_t CLS_NARROW = 0, CLS_WIDE = 1, CLS_HASH1 = 2, CLS_HASH2 = 3;
struct QueueState {
    uint32_t bcount[NCLASS][NBUCKET];
    uint32_t cursor[NCLASS][NBUCKET];
    uint32_t n_items[NCLASS];
    uint32_t head[NCLASS];              // next item to hand out
    uint32_t done[NCLASS];              // workgroups finished
    uint32_t ovf_count, ovf_head;       // hash starts handed back to the narrow walk
    unsigned long long acc;             // running total of the count
};

// Wedges of start u: sum over v in N(u) of the entries of adj_B[v] after u
// (all entries but u itself when `all_ends`, for the local counts).
// Bucket = bit length of that count (0 = nothing to do); class 1 = wide.
// Class: wide when d_u > narrow_max, else hash when the wedges fit the
// small (<= hs_max) or mid (<= hm_max) tables, else narrow.  With split != 0
// (local counts) a start of more than `split` wedges is wide too, and a wide
// start is cut into ceil(wedges / split) parts (at most one per table window
// and SPLIT_MAX), each an item of its own (nsplit[u] parts).
// A narrow start takes a hash table only when it is sparse: at most
// hl.density wedges (default HASH_DENSITY) per counter window its end points
// span (the window walk pays about one round trip per window it touches).
// A start of at most half_density wedges per spanned window is marked
// (bucket bit 15) for the narrow walk's short pieces, one of at most
// QUARTER_DENSITY (bucket bit 14) for its shortest.
constexpr uint64_t SPLIT_WEDGES = 1ull << 24;  // local counts: wedges per part of a wide start
constexpr uint32_t SPLIT_MAX = 4096;
constexpr uint32_t HASH_DENSITY = 32, HALF_DENSITY = 384, QUARTER_DENSITY = 128;
constexpr uint16_t BUCKET_SPARSE = 0x8000, BUCKET_SPARSER = 0x4000;
__global__ __launch_bounds__(256) void k_work(const uint32_t *offA, const uint32_t *adjA,
                                              const uint32_t *xA, const uint32_t *offB,
                                              const uint32_t *adjB,
                                              uint32_t nA, int all_ends, const uint8_t *mark,
                                              uint32_t narrow_max, uint32_t hs_max,
                                              uint32_t hm_max, uint32_t density,
                                              uint32_t half_density, uint64_t split,
                                              uint16_t *bucket, uint16_t *nsplit,
                                              QueueState *q) {
    __shared__ uint32_t hist[NCLASS][NBUCKET];
    for (int i = threadIdx.x; i < NCLASS * NBUCKET; i += blockDim.x) (&hist[0][0])[i] = 0;
    __syncthreads();
    const int lane = threadIdx.x & (WAVE - 1);
    const uint32_t wpb = blockDim.x / WAVE;
    for (uint32_t u = blockIdx.x * wpb + threadIdx.x / WAVE; u < nA; u += gridDim.x * wpb) {
        uint32_t rb = offA[u], re = offA[u + 1];
        if (mark && !mark[u]) re = rb;          // start not asked for
        unsigned long long t = 0;
        uint32_t top = 0;                       // highest end point rank
        const bool spans = (hs_max | hm_max | half_density) != 0u;
        for (uint32_t k = rb + lane; k < re; k += WAVE) {
            uint32_t v = adjA[k];
            const uint32_t e = offB[v + 1];
            t += e - (all_ends ? offB[v] : xA[k]) - 1;
            if (spans) top = max(top, adjB[e - 1]);
        }
        t = wave_sum64(t);
        top = wave_incl_max(top);
        top = wave_last(top);
        // lowest end point rank: above u for the exact count; the local
        // counts take all end points, whose span is taken from rank 0
        const uint32_t bot = all_ends ? 0u : u;
        // a start with one midpoint shares at most one with any w: C_u[w] <= 1
        // adds nothing to a count, so it is not queued (its outputs stay 0)
        if (re - rb < 2) t = 0;
        if (lane == 0) {
            uint32_t b = t ? 64 - __clzll(t) : 0;
            const uint32_t span = top >= bot ? (top >> G_SHIFT) - (bot >> G_SHIFT) + 1 : 1u;
            const bool spread = t <= (uint64_t)density * span;
            const bool sparse = t <= (uint64_t)half_density * span;
            // with split, a start of more than one part's wedges takes the wide
            // kernel (whatever its degree), so that its parts can run side by side
            uint32_t cls = ((re - rb) > narrow_max || (split && t > split)) ? CLS_WIDE
                         : !spread ? CLS_NARROW
                         : t <= hs_max ? CLS_HASH1 : t <= hm_max ? CLS_HASH2 : CLS_NARROW;
            uint32_t G = 1;
            if (cls == CLS_WIDE && split) {
                const uint32_t logw = (re - rb) <= 0xFFFFu ? 1u : 0u;
                const uint64_t nwin = ((nA - 1) >> (G_SHIFT + logw)) + 1;
                uint64_t gg = (t + split - 1) / split;
                gg = gg < nwin ? gg : nwin;
                gg = gg < SPLIT_MAX ? gg : SPLIT_MAX;
                G = gg > 1 ? (uint32_t)gg : 1u;
            }
            const bool sparser = half_density && t <= (uint64_t)QUARTER_DENSITY * span;
            bucket[u] = (uint16_t)(b | cls << 8) | (sparse ? BUCKET_SPARSE : 0) |
                        (sparser ? BUCKET_SPARSER : 0);
            if (nsplit) nsplit[u] = (uint16_t)G;
            if (b) atomicAdd(&hist[cls][b], G);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < NCLASS * NBUCKET; i += blockDim.x)
        if ((&hist[0][0])[i]) atomicAdd(&(&q->bcount[0][0])[i], (&hist[0][0])[i]);
}

// Bucket b's items start after all larger buckets (largest work first).
__global__ void k_bucket_offsets(QueueState *q) {
    if (threadIdx.x < NCLASS) {
        const int c = threadIdx.x;
        uint32_t run = 0;
        for (int b = NBUCKET - 1; b >= 1; b--) {
            q->cursor[c][b] = run;
            run += q->bcount[c][b];
        }
        q->n_items[c] = run;
        q->head[c] = 0;
        q->done[c] = 0;
    }
    if (threadIdx.x == 0) {
        q->acc = 0;
        q->ovf_count = 0;
        q->ovf_head = 0;
    }
}

struct ItemLists {
    uint32_t *l[NCLASS];
    uint32_t *wide_g;             // part g | parts << 16 of each wide item
    const uint16_t *nsplit;       // parts of each start (NULL: one)
};

__global__ __launch_bounds__(256) void k_scatter_items(const uint16_t *bucket, uint32_t nA,
                                                       QueueState *q, ItemLists items) {
    __shared__ uint32_t hist[NCLASS][NBUCKET], base[NCLASS][NBUCKET];
    // blocks stride over chunks of blockDim.x starts (the grid is capped)
    for (uint64_t c0 = (uint64_t)blockIdx.x * blockDim.x; c0 < nA;
         c0 += (uint64_t)gridDim.x * blockDim.x) {
        for (int i = threadIdx.x; i < NCLASS * NBUCKET; i += blockDim.x) (&hist[0][0])[i] = 0;
        __syncthreads();
        const uint64_t u = c0 + threadIdx.x;
        uint32_t b = 0, cls = 0, local = 0, G = 1;
        if (u < nA) {
            b = bucket[u] & 255u;
            cls = (bucket[u] >> 8) & (NCLASS - 1);
            if (cls == CLS_WIDE && items.nsplit) G = items.nsplit[u];
            if (b) local = atomicAdd(&hist[cls][b], G);
        }
        __syncthreads();
        for (int i = threadIdx.x; i < NCLASS * NBUCKET; i += blockDim.x) {
            uint32_t h = (&hist[0][0])[i];
            if (h) (&base[0][0])[i] = atomicAdd(&(&q->cursor[0][0])[i], h);
        }
        __syncthreads();
        if (b) {
            for (uint32_t g = 0; g < G; g++) {
                const uint32_t at = base[cls][b] + local + g;
                items.l[cls][at] = (uint32_t)u;
                if (cls == CLS_WIDE) items.wide_g[at] = g | G << 16;
            }
        }
        __syncthreads();            // hist and base are reset for the next chunk
    }
}

__global__ void k_zero_u32(uint32_t *p, uint64_t n) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

__global__ void k_zero_u64(unsigned long long *p, uint64_t n) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// End of a persistent launch over class `cls`: add this workgroup's sum; the
// last workgroup to finish re-arms the class's queue for the next launch and,
// when `total` is given, publishes the count and clears the accumulator.
__device__ inline void finish_launch(QueueState *q, int cls, unsigned long long part,
                                     unsigned long long *total) {
    if (threadIdx.x != 0) return;
    if (part) atomicAdd(&q->acc, part);
    __threadfence();
    uint32_t d = atomicAdd(&q->done[cls], 1u);
    if (d == gridDim.x - 1) {
        __threadfence();
        if (total) {
            *total = atomicAdd(&q->acc, 0ull);
            q->acc = 0;
        }
        q->head[cls] = 0;
        q->done[cls] = 0;
        if (cls == (int)CLS_NARROW) {       // the narrow launch drained the overflow list
            q->ovf_count = 0;
            q->ovf_head = 0;
        }
        __threadfence();
    }
}

struct CountArgs {
    const uint32_t *offA, *adjA, *xA, *offB, *adjB;
    const uint32_t *seg1, *seg_start, *seg_win;
    const uint32_t *items, *items_wide, *items_h1, *items_h2;
    uint32_t *ovf;                      // hash starts handed back to the narrow walk
    const uint16_t *bucket;             // per start: work bucket, class, BUCKET_SPARSE
    QueueState *q;
    uint32_t nA;
    uint32_t chunk;                     // narrow starts per queue access
    uint32_t hash_passes;               // passes of a hash start (0: from its wedges)
    unsigned long long *total;
    unsigned long long *per_start;      // butterflies found from each start (rank), or null
};

// Local counts.  For a start u the walk takes every endpoint w != u (no
// order), so C_u[w] = |N(u) & N(w)| for all same-side w and
//   B_u       = sum_w C(C_u[w], 2)                       (Eq. (2))
//   B_(u,v)   = sum_{w in N(v), w != u} (C_u[w] - 1)       (edge definition)
//   B_v (mid) = 1/2 sum_{u in N(v)} B_(u,v)               (two edges of v per butterfly)
// After a window's increments the final counts of its entries are read again
// and summed per midpoint.
struct LocalArgs {
    CountArgs c;
    const uint32_t *eidA, *idA;
    unsigned long long *cntA;     // per start-side vertex (caller ids), or null
    unsigned long long *cntE;     // per edge (caller order), or null
    unsigned long long *epos;     // B_(u,v) by A-side adjacency position (workspace), or null
    int pass2;                    // edge / midpoint sums wanted (else B_u only)
    // wide starts split over several workgroups: item it covers part
    // wide_g[it] & 0xFFFF of wide_g[it] >> 16 (equal runs of table windows);
    // a split start's parts add into esum_g (per adjacency position) and the
    // last part to finish (wdone[u]) writes its edges
    const uint32_t *wide_g;
    uint32_t *wdone;
    unsigned long long *esum_g;
};

// Per-midpoint state of wide starts, one slot per A-side adjacency position.
// Indexed by the start's adjacency position k, or, with stride != 0, by
// blockIdx.x * stride + the midpoint's index j (one slice per workgroup,
// so several workgroups can walk parts of one start).
struct WideScratch {
    uint32_t *pos, *seg;          // cursor: next position and its segment
    uint32_t *lim, *sw, *se;      // list end; window and end of the cursor's segment
    uint32_t *lo, *hi;            // sub-run of the current window (local counts)
    unsigned long long *esum;     // sums of final counts (local counts)
    uint64_t stride;
    __device__ inline uint64_t at(uint32_t j, uint32_t k) const {
        return stride ? blockIdx.x * stride + j : k;
    }
};

// Per-edge and per-midpoint output of one (start, midpoint) pair.
__device__ inline void emit_edge(const LocalArgs &a, uint32_t k, uint32_t v, uint32_t dv,
                                 unsigned long long s) {
    (void)v;
    const unsigned long long e = s - (unsigned long long)(dv - 1);
    if (a.cntE) a.cntE[a.eidA[k]] = e;
    if (a.epos) a.epos[k] = e;
}

// A group: 4 consecutive adjacency entries at `base` (16-byte aligned), of
// which those in [lo, hi) other than `skip` belong to the sub-run.
__device__ inline uint32_t group_mask(uint32_t base, uint32_t lo, uint32_t hi, uint32_t skip) {
    uint32_t m = 0;
#pragma unroll
    for (int i = 0; i < 4; i++) {
        uint32_t pos = base + i;
        m |= (uint32_t)(pos >= lo && pos < hi && pos != skip) << i;
    }
    return m;
}

// ------------------------------------------------------------------ narrow: one wave per start
// A window's sub-runs are cut into pieces of WK consecutive groups (16
// entries) of one midpoint; lanes take pieces round-robin, so one search maps
// a piece to its midpoint and the entries of a piece are contiguous.  The
// narrow walk of a start whose windows are sparse (few wedges per window its
// end points span, marked by the plan) cuts pieces of WK_SPARSE groups, and
// of one group for the sparsest starts of the exact count: a window's work
// is then spread over more lanes and each lane's counter updates (whose
// cost does not depend on how many of its entries are in the sub-run) are
// halved or quartered.
constexpr int WK = 4, WK_SPARSE = 2;

template <bool LOCAL>
struct WShared {
    uint32_t tbl[WTBL_WORDS + WT];      // byte counters, then one zero word per lane
    uint32_t pre[WSLOTS * WT];          // exclusive prefix of pieces per midpoint
    uint32_t lo[WSLOTS * WT], hi[WSLOTS * WT];
    uint32_t own[WT];                   // 1 + midpoint of piece i (windows of <= 64 pieces)
    uint32_t skip[LOCAL ? WSLOTS * WT : 1];
    unsigned long long esum[LOCAL ? WSLOTS * WT : 1];
};

// One lane's piece: entries base .. base + 4*WK - 1, of which those with
// pos - lo < len (and pos != skip) are in the sub-run.
struct Piece {
    uint32_t base, lo, len, skip, j;
};

template <bool LOCAL, int K = WK>
__device__ inline Piece wpiece(const WShared<LOCAL> &sh, uint32_t du, uint32_t pi, bool valid) {
    // branch-free search over the du midpoint prefixes (uniform trip count)
    uint32_t j = 0;
    for (uint32_t s = 1u << (31 - __clz(du)); s; s >>= 1) {
        const uint32_t t = j + s;
        const uint32_t pv = sh.pre[(t <= du ? t : du) - 1];
        j = (t <= du && pv <= pi) ? t : j;
    }
    j -= 1;
    Piece pc;
    const uint32_t lo = sh.lo[j], hi = sh.hi[j];
    const uint32_t g0 = (lo >> 2) + (pi - sh.pre[j]) * K;
    const uint32_t end = min(hi, (g0 + K) << 2);
    pc.base = valid ? g0 << 2 : 0;
    pc.lo = lo;
    pc.len = valid ? end - lo : 0;
    pc.skip = LOCAL ? sh.skip[j] : INF;
    pc.j = j;
    return pc;
}

// Piece `lane` of a window with at most one piece per lane: the owner
// table holds 1 + midpoint at each midpoint's first piece; a wave max-scan
// carries it over that midpoint's other pieces (midpoints and their first
// pieces increase together).
template <bool LOCAL, int K = WK>
__device__ inline Piece wpiece_direct(const WShared<LOCAL> &sh, uint32_t lane, bool valid) {
    const uint32_t o = wave_incl_max(sh.own[lane]);
    const uint32_t j = min((o ? o : 1u) - 1, (uint32_t)(WSLOTS * WT - 1));
    Piece pc;
    const uint32_t lo = sh.lo[j], hi = sh.hi[j];
    const uint32_t g0 = (lo >> 2) + (lane - sh.pre[j]) * K;
    const uint32_t end = min(hi, (g0 + K) << 2);
    pc.base = valid ? g0 << 2 : 0;
    pc.lo = lo;
    pc.len = valid ? end - lo : 0;
    pc.skip = LOCAL ? sh.skip[j] : INF;
    pc.j = j;
    return pc;
}

template <int N>
__device__ inline void wfetch(const uint32_t *adjB, const Piece &pc, uint4 *q) {
#pragma unroll
    for (int k = 0; k < N; k++) q[k] = *(const uint4 *)(adjB + pc.base + 4 * k);
}

// Bit i set when entry base + i of an N-entry piece is in the sub-run
// [lo, lo + len) and is not `skip` (computed once per piece, so that each
// entry tests one bit).  A piece of a sub-run starts at most three entries
// before lo and ends inside the run, so 0 <= lo - base < end - base <= N.
template <bool LOCAL, int N>
__device__ inline uint32_t piece_bits(const Piece &pc) {
    const uint32_t a = pc.lo > pc.base ? pc.lo - pc.base : 0u;
    const uint32_t e = pc.lo + pc.len - pc.base;
    uint32_t m = pc.len ? ((1u << e) - 1u) & ~((1u << a) - 1u) : 0u;
    if (LOCAL) {
        const uint32_t d = pc.skip - pc.base;
        m &= d < (uint32_t)N ? ~(1u << d) : ~0u;
    }
    return m;
}

// Entry i of the piece -> byte offset of its counter, or of the lane's zero
// word when it is not in the sub-run (bit i of m clear).
__device__ inline uint32_t wslot(uint32_t m, uint32_t i, uint32_t w, uint32_t wb,
                                 uint32_t zero_byte) {
    return (m >> i) & 1u ? w - wb : zero_byte;
}

// Add one to every counter of the piece; the counters' previous values are
// what the pairs gain.  A zero word gets a zero increment and returns zero.
// NIB: 4-bit counters (starts of degree <= 15, so C_u[w] <= 15 and an
// increment never carries into the next counter), eight per word; entry
// slots are then nibble indices and the zero word is nibbles 8 z .. 8 z + 7.
template <bool LOCAL, bool NIB = false, int K = WK>
__device__ inline uint32_t wbump(WShared<LOCAL> &sh, const Piece &pc, const uint4 *q, uint32_t wb) {
    constexpr uint32_t PER = NIB ? 8 : 4, LOGP = NIB ? 3 : 2, BITS = NIB ? 4 : 8;
    const uint32_t zb = (WTBL_WORDS + threadIdx.x) * PER;
    const uint32_t m = piece_bits<LOCAL, 4 * K>(pc);
    uint32_t old[4 * K], sft[4 * K];
#pragma unroll
    for (int k = 0; k < K; k++) {
        const uint32_t w[4] = {q[k].x, q[k].y, q[k].z, q[k].w};
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const bool on = (m >> (4 * k + i)) & 1u;
            const uint32_t b = on ? w[i] - wb : zb;
            // the counter's bit offset, (b mod PER) * BITS, is the low five
            // bits of b * BITS: shifts and field extracts read only those
            const uint32_t sb = b * BITS;
            sft[4 * k + i] = sb;
            old[4 * k + i] = atomicAdd(&sh.tbl[b >> LOGP], on ? 1u << (sb & 31u) : 0u);
        }
    }
    // Keep the extraction below the sixteen atomics so that they are all in
    // flight before the first result is waited for: an empty volatile asm
    // that takes each result (no instruction is emitted).
#pragma unroll
    for (int k = 0; k < 4 * K; k++) asm volatile("" : "+v"(old[k]));
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < 4 * K; k++) s += __builtin_amdgcn_ubfe(old[k], sft[k], BITS);
    return s;
}

// Sum of the counters of the piece's entries.
template <bool LOCAL, bool NIB = false, int K = WK>
__device__ inline uint32_t wread(const WShared<LOCAL> &sh, const Piece &pc, const uint4 *q,
                                 uint32_t wb) {
    const uint8_t *t8 = (const uint8_t *)sh.tbl;
    const uint32_t zb = (WTBL_WORDS + threadIdx.x) * (NIB ? 8 : 4);
    const uint32_t m = piece_bits<LOCAL, 4 * K>(pc);
    uint32_t v[4 * K];
#pragma unroll
    for (int k = 0; k < K; k++) {
        const uint32_t w[4] = {q[k].x, q[k].y, q[k].z, q[k].w};
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const uint32_t b = wslot(m, 4 * k + i, w[i], wb, zb);
            v[4 * k + i] = NIB ? (sh.tbl[b >> 3] >> ((b & 7u) * 4)) & 0xFu : t8[b];
        }
    }
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < 4 * K; k++) s += v[k];
    return s;
}

// Clear the piece's counters (nibbles: an atomic and, since other lanes may
// clear the word's other nibbles at the same time).
template <bool LOCAL, bool NIB = false, int K = WK>
__device__ inline void wclear(WShared<LOCAL> &sh, const Piece &pc, const uint4 *q, uint32_t wb) {
    uint8_t *t8 = (uint8_t *)sh.tbl;
    const uint32_t zb = (WTBL_WORDS + threadIdx.x) * (NIB ? 8 : 4);
    const uint32_t m = piece_bits<LOCAL, 4 * K>(pc);
#pragma unroll
    for (int k = 0; k < K; k++) {
        const uint32_t w[4] = {q[k].x, q[k].y, q[k].z, q[k].w};
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const uint32_t b = wslot(m, 4 * k + i, w[i], wb, zb);
            if (NIB) atomicAnd(&sh.tbl[b >> 3], ~(0xFu << ((b & 7u) * 4)));
            else t8[b] = 0;
        }
    }
}

template <bool LOCAL>
__device__ inline void wclear_all(WShared<LOCAL> &sh) {
    const uint4 z = make_uint4(0, 0, 0, 0);
#pragma unroll
    for (int i = 0; i < WTBL_BYTES / 16 / WT; i++) ((uint4 *)sh.tbl)[i * WT + threadIdx.x] = z;
}

// Walk of one narrow start by one wave.  Lane l owns midpoints l + 64 s.
// EXACT: endpoints ranked above u.  LOCAL: all endpoints other than u, with
// the per-midpoint sums of final counts accumulated in sh.esum.
// In a workgroup of one wave the LDS operations execute in issue order, so
// ordering them needs only a compiler barrier (no wait for completion).
__device__ inline void wave_order() { __builtin_amdgcn_wave_barrier(); }

// Order this wave's LDS writes before its later reads (no other wave involved).
__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// NIB: the 4-bit table covers 2^15 ranks (two segment windows); a slot's
// sub-run of a table window is then one segment or two consecutive ones, so
// the slot looks two segments ahead (w2/s2, w3/s3).  Windows are indexed in
// table units (segment window >> LOGW).
template <bool LOCAL, bool NIB, int K>
__device__ unsigned long long wave_walk(const CountArgs &a, WShared<LOCAL> &sh, uint32_t rb,
                                        uint32_t du, bool pass2) {
    constexpr int LOGW = NIB ? 1 : 0;
    const uint32_t lane = threadIdx.x;
    const uint32_t ns = (du + WT - 1) / WT;
    uint32_t p[WSLOTS], ev[WSLOTS], cur[WSLOTS], win[WSLOTS], sn[WSLOTS], w2[WSLOTS], s2[WSLOTS];
    uint32_t w3[WSLOTS], s3[WSLOTS];
#pragma unroll
    for (int s = 0; s < WSLOTS; s++) {
        p[s] = ev[s] = cur[s] = sn[s] = s2[s] = s3[s] = 0;
        win[s] = w2[s] = w3[s] = INF;
        uint32_t skip = INF;
        const uint32_t j = lane + s * WT;
        if (s < (int)ns && j < du) {
            const uint32_t k = rb + j;
            const uint32_t v = a.adjA[k];
            const uint32_t x = a.xA[k];
            const uint32_t pb = a.offB[v];
            ev[s] = a.offB[v + 1];
            p[s] = LOCAL ? pb : x + 1;
            if (LOCAL) skip = x;
            if (LOCAL ? (ev[s] - pb > 1) : (p[s] < ev[s])) {
                cur[s] = a.seg1[p[s]] - 1;
                win[s] = a.seg_win[cur[s]] >> LOGW;
                sn[s] = a.seg_start[cur[s] + 1];
                if (sn[s] < ev[s]) {
                    w2[s] = a.seg_win[cur[s] + 1] >> LOGW;
                    s2[s] = a.seg_start[cur[s] + 2];
                    if (NIB && s2[s] < ev[s]) {
                        w3[s] = a.seg_win[cur[s] + 2] >> LOGW;
                        s3[s] = a.seg_start[cur[s] + 3];
                    }
                }
            }
        }
        if (LOCAL) {
            sh.skip[j] = skip;
            sh.esum[j] = 0;
        }
    }
    // Advance every slot past the current window, publish the sub-runs of
    // the next window touched (kw, INF when none), their piece prefix and,
    // for a window of at most one piece per lane, the owner table; returns
    // the number of pieces.
    uint32_t first[WSLOTS], cnt[WSLOTS];  // this lane's midpoints: first piece, pieces
    auto next_window = [&](uint32_t &kw) -> uint32_t {
        uint32_t mn = INF;
#pragma unroll
        for (int s = 0; s < WSLOTS; s++) mn = min(mn, win[s]);
        kw = wave_min(mn);
        if (kw == INF) return 0u;
        uint32_t run = 0;
#pragma unroll
        for (int s = 0; s < WSLOTS; s++) first[s] = cnt[s] = 0;
#pragma unroll
        for (int s = 0; s < WSLOTS; s++) {
            if (s >= (int)ns) break;
            // branch-free: the look-ahead loads below must not be merged at
            // a branch join (that would wait for them here)
            const bool act = win[s] == kw;
            const uint32_t h1 = sn[s] < ev[s] ? sn[s] : ev[s];
            // NIB: the next segment (inside the list) in the same table window
            const bool two = NIB && act && h1 < ev[s] && w2[s] == kw;
            const uint32_t h = two ? (s2[s] < ev[s] ? s2[s] : ev[s]) : h1;
            const uint32_t lo = act ? p[s] : 0u, hi = act ? h : 0u;
            const uint32_t np = act ? (((hi + 3) >> 2) - (lo >> 2) + K - 1) / K : 0u;
            const bool adv = act && h < ev[s];
            p[s] = act ? h : p[s];
            cur[s] += adv ? (two ? 2u : 1u) : 0u;
            // bitwise blends rather than selects between the look-ahead
            // registers (a select of two array elements can be turned into a
            // load through a selected address, which keeps the arrays in
            // scratch memory)
            const uint32_t tm = 0u - (uint32_t)two;
            const uint32_t nw = w2[s] ^ ((w2[s] ^ w3[s]) & tm);
            const uint32_t ne = s2[s] ^ ((s2[s] ^ s3[s]) & tm);
            win[s] = act ? (adv ? nw : INF) : win[s];
            sn[s] = adv ? ne : sn[s];
            // look-ahead from the cursor (unchanged values when it did not
            // move); used from the next window on.  cur + 3 <= segments + 2,
            // inside the padded segment arrays.
            w2[s] = a.seg_win[cur[s] + 1] >> LOGW;
            s2[s] = a.seg_start[cur[s] + 2];
            if (NIB) {
                w3[s] = a.seg_win[cur[s] + 2] >> LOGW;
                s3[s] = a.seg_start[cur[s] + 3];
            }
            const uint32_t inc = wave_incl_scan(np);
            const uint32_t j = lane + s * WT;
            sh.pre[j] = run + inc - np;
            sh.lo[j] = lo;
            sh.hi[j] = hi;
            first[s] = run + inc - np;
            cnt[s] = np;
            run += wave_last(inc);
        }
        if (run <= (uint32_t)WT) {
            sh.own[lane] = 0;
            wave_order();
#pragma unroll
            for (int s = 0; s < WSLOTS; s++)
                if (cnt[s]) sh.own[first[s]] = lane + s * WT + 1;
        }
        return run;
    };

    // Bump, second look and clear of one window held in registers.
    auto finish = [&](const Piece &pc, const uint4 *q, uint32_t wb) -> uint32_t {
        const uint32_t part = wbump<LOCAL, NIB, K>(sh, pc, q, wb);
        if (LOCAL && pass2) {
            wave_order();
            const uint32_t v = wread<LOCAL, NIB, K>(sh, pc, q, wb);
            if (v) atomicAdd(&sh.esum[pc.j], (unsigned long long)v);
        }
        wave_order();
        wclear<LOCAL, NIB, K>(sh, pc, q, wb);
        wave_order();
        return part;
    };

    // Windows of at most one piece per lane run as a two-stage pipeline: the
    // pieces of the next window are loaded while the current window's
    // counters are bumped and cleared.  The loop is unrolled twice so that
    // the two register buffers swap roles without a copy (a copy would wait
    // for the loads in flight).  A window with more pieces than lanes is
    // walked in rounds from the published prefixes.
    unsigned long long sum = 0;
    uint32_t kw;                        // the published window
    uint32_t NP = next_window(kw);
    wave_order();
    Piece pa, pb;
    uint4 qa[K], qb[K];
    while (kw != INF) {
        if (NP > (uint32_t)WT) {
            // Rounds of 64 pieces.  Round r's pieces are mapped to midpoints
            // through the owner table (the midpoints whose first piece falls
            // in the round, plus the one carried over from the round
            // before), and the next round's pieces are loaded while this
            // round's counters are bumped (unrolled twice, no copies).
            const uint32_t wb = kw << (G_SHIFT + LOGW);
            const uint32_t rounds = (NP + WT - 1) / WT;
            auto map_round = [&](uint32_t r, uint32_t &carry) -> Piece {
                const uint32_t r0 = r * WT;
                sh.own[lane] = 0;
                wave_order();
#pragma unroll
                for (int s = 0; s < WSLOTS; s++)
                    if (cnt[s] && first[s] - r0 < (uint32_t)WT)
                        sh.own[first[s] - r0] = lane + s * WT + 1;
                wave_order();
                const uint32_t o = max(wave_incl_max(sh.own[lane]), carry);
                carry = wave_last(o);
                const uint32_t j = min((o ? o : 1u) - 1, (uint32_t)(WSLOTS * WT - 1));
                const uint32_t pi = r0 + lane;
                const bool valid = pi < NP;
                Piece pc;
                const uint32_t lo = sh.lo[j], hi = sh.hi[j];
                const uint32_t g0 = (lo >> 2) + (pi - sh.pre[j]) * K;
                const uint32_t end = min(hi, (g0 + K) << 2);
                pc.base = valid ? g0 << 2 : 0;
                pc.lo = lo;
                pc.len = valid ? end - lo : 0;
                pc.skip = LOCAL ? sh.skip[j] : INF;
                pc.j = j;
                return pc;
            };
            // pass 0 bumps the counters, pass 1 reads the final counts
            for (int pass = 0; pass < ((LOCAL && pass2) ? 2 : 1); pass++) {
                uint32_t carry = 0, part = 0;
                Piece r0p = map_round(0, carry);
                uint4 q0[K], q1[K];
                wfetch<K>(a.adjB, r0p, q0);
                for (uint32_t r = 0;; r += 2) {
                    Piece r1p = map_round(r + 1, carry);
                    wfetch<K>(a.adjB, r1p, q1);
                    if (pass == 0) {
                        part += wbump<LOCAL, NIB, K>(sh, r0p, q0, wb);
                    } else {
                        const uint32_t v = wread<LOCAL, NIB, K>(sh, r0p, q0, wb);
                        if (v) atomicAdd(&sh.esum[r0p.j], (unsigned long long)v);
                    }
                    if (r + 1 >= rounds) break;
                    r0p = map_round(r + 2, carry);
                    wfetch<K>(a.adjB, r0p, q0);
                    if (pass == 0) {
                        part += wbump<LOCAL, NIB, K>(sh, r1p, q1, wb);
                    } else {
                        const uint32_t v = wread<LOCAL, NIB, K>(sh, r1p, q1, wb);
                        if (v) atomicAdd(&sh.esum[r1p.j], (unsigned long long)v);
                    }
                    if (r + 2 >= rounds) break;
                }
                sum += part;
                wave_order();            // every count of the window is final
            }
            wclear_all(sh);
            wave_order();
            NP = next_window(kw);
            wave_order();
            continue;
        }
        // prologue: window kw into (pa, qa), publish the following one
        pa = wpiece_direct<LOCAL, K>(sh, lane, lane < NP);
        wfetch<K>(a.adjB, pa, qa);
        uint32_t kwa = kw;
        wave_order();
        NP = next_window(kw);
        wave_order();
        for (;;) {
            // (pa, qa) hold window kwa; window kw is published
            // the next window's loads are issued unconditionally (a lane
            // without a piece reads the first group) so that no branch
            // joins the buffers while their loads are in flight
            bool more = kw != INF && NP <= (uint32_t)WT;
            pb = wpiece_direct<LOCAL, K>(sh, lane, more && lane < NP);
            wfetch<K>(a.adjB, pb, qb);
            sum += finish(pa, qa, kwa << (G_SHIFT + LOGW));
            if (!more) break;
            const uint32_t kwb = kw;
            NP = next_window(kw);
            wave_order();
            // (pb, qb) hold window kwb; window kw is published
            more = kw != INF && NP <= (uint32_t)WT;
            pa = wpiece_direct<LOCAL, K>(sh, lane, more && lane < NP);
            wfetch<K>(a.adjB, pa, qa);
            sum += finish(pb, qb, kwb << (G_SHIFT + LOGW));
            if (!more) break;
            kwa = kw;
            NP = next_window(kw);
            wave_order();
        }
        // here window kw (if any) has more pieces than lanes, or none is left
    }
    return sum;
}

// Hand out `chunk` starts per queue access.
__device__ inline uint32_t wave_take(QueueState *q, int cls, uint32_t chunk) {
    uint32_t b = 0;
    if (threadIdx.x == 0) b = atomicAdd(&q->head[cls], chunk);
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)b);
}

__device__ inline uint32_t wave_take_ovf(QueueState *q) {
    uint32_t b = 0;
    if (threadIdx.x == 0) b = atomicAdd(&q->ovf_head, 1u);
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)b);
}

__global__ __launch_bounds__(WT) void k_exact_narrow(CountArgs a) {
    __shared__ WShared<false> sh;
    wclear_all(sh);
    sh.tbl[WTBL_WORDS + threadIdx.x] = 0;
    __syncthreads();
    unsigned long long acc = 0;
    const uint32_t n = a.q->n_items[CLS_NARROW];
    // the class's queue first, then the starts the hash kernels (launched
    // before this one) handed back; one walk site keeps the code small
    bool ovf = false;
    uint32_t no = 0;
    uint32_t b = wave_take(a.q, CLS_NARROW, a.chunk);
    uint32_t e = b < n ? min(b + a.chunk, n) : b;
    for (;;) {
        if (b >= e) {
            if (!ovf) {
                b = wave_take(a.q, CLS_NARROW, a.chunk);
                e = b < n ? min(b + a.chunk, n) : b;
                if (b >= n) {
                    ovf = true;
                    no = a.q->ovf_count;
                }
            }
            if (ovf) {
                b = wave_take_ovf(a.q);
                e = b + 1;
                if (b >= no) break;
            }
        }
        const uint32_t u = ovf ? a.ovf[b] : a.items[b];
        b++;
        const uint32_t rb = a.offA[u];
        const uint32_t du = a.offA[u + 1] - rb;
        const uint16_t bk = a.bucket[u];
        const bool sp = (bk & BUCKET_SPARSE) != 0, sp2 = (bk & BUCKET_SPARSER) != 0;
        const unsigned long long s =
            du <= 15u ? (sp2 ? wave_walk<false, true, 1>(a, sh, rb, du, false)
                         : sp ? wave_walk<false, true, WK_SPARSE>(a, sh, rb, du, false)
                              : wave_walk<false, true, WK>(a, sh, rb, du, false))
                      : (sp2 ? wave_walk<false, false, 1>(a, sh, rb, du, false)
                         : sp ? wave_walk<false, false, WK_SPARSE>(a, sh, rb, du, false)
                              : wave_walk<false, false, WK>(a, sh, rb, du, false));
        if (a.per_start) {
            const unsigned long long t = wave_sum64(s);
            if (threadIdx.x == 0) a.per_start[u] = t;
        }
        acc += s;
    }
    acc = wave_sum64(acc);
    finish_launch(a.q, CLS_NARROW, acc, nullptr);
}

__global__ __launch_bounds__(WT) void k_local_narrow(LocalArgs a) {
    __shared__ WShared<true> sh;
    wclear_all(sh);
    sh.tbl[WTBL_WORDS + threadIdx.x] = 0;
    __syncthreads();
    const uint32_t n = a.c.q->n_items[0];
    for (uint32_t b = wave_take(a.c.q, 0, a.c.chunk); b < n; b = wave_take(a.c.q, 0, a.c.chunk)) {
        const uint32_t e = b + a.c.chunk < n ? b + a.c.chunk : n;
        for (uint32_t it = b; it < e; it++) {
            const uint32_t u = a.c.items[it];
            const uint32_t rb = a.c.offA[u], du = a.c.offA[u + 1] - rb;
            const bool sp = (a.c.bucket[u] & BUCKET_SPARSE) != 0;
            unsigned long long s =
                du <= 15u ? (sp ? wave_walk<true, true, WK_SPARSE>(a.c, sh, rb, du, a.pass2)
                                : wave_walk<true, true, WK>(a.c, sh, rb, du, a.pass2))
                          : (sp ? wave_walk<true, false, WK_SPARSE>(a.c, sh, rb, du, a.pass2)
                                : wave_walk<true, false, WK>(a.c, sh, rb, du, a.pass2));
            if (a.pass2) {
                for (uint32_t j = threadIdx.x; j < du; j += WT) {
                    const uint32_t k = rb + j;
                    const uint32_t v = a.c.adjA[k];
                    emit_edge(a, k, v, a.c.offB[v + 1] - a.c.offB[v], sh.esum[j]);
                }
            }
            s = wave_sum64(s);
            if (threadIdx.x == 0 && a.cntA) a.cntA[a.idA[u]] = s;
            __syncthreads();
        }
    }
    finish_launch(a.c.q, 0, 0, nullptr);
}

// ------------------------------------------------------------------ hash: sparse starts
// A start with few wedges for the span of ranks they reach crosses many
// nearly empty windows, each a round trip of the window walk.  Such a start
// keeps C_u[w] in an LDS hash table instead and walks its midpoints' whole
// suffixes in one pass: key w + 1 (0 = empty) placed by multiplicative
// hashing with double hashing, a byte counter beside it (C_u[w] <= d_u <=
// 255).  A compare-and-swap claims or finds the key, and the counter's old
// value is what the pair {u, w} gains, as in the window walk.  A start with
// more wedges than half the table takes several passes, each over the end
// points of one hash partition (the table is cleared between passes).  A
// pass that fills the table (only possible when a partition gets more than
// twice its share) gives the start back to the narrow window walk, which
// counts it from scratch.
// Small table: one wave per start; mid table: a workgroup of four waves.
constexpr int HS_SLOTS = 1024, HM_SLOTS = 8192;
constexpr uint32_t HS_CAP = HS_SLOTS / 2, HM_CAP = HM_SLOTS / 2;   // entries per pass
constexpr uint32_t HASH_PASSES = 4;
constexpr uint32_t HS_MAX = HASH_PASSES * HS_CAP, HM_MAX = HASH_PASSES * HM_CAP;
// default wedge limit of the small table (the mid table takes the starts above it)
constexpr uint32_t HS_DEFAULT = 1024;
constexpr uint32_t HASH_FULL = 0xFFFFFFFFu;

template <int NW, int S>
struct HShared {
    uint32_t key[S];                    // w + 1, 0 = empty
    uint32_t cnt[S / 4];                // byte counters, four per word
    uint32_t zero[64 * NW];             // one word per thread that stays 0
    uint32_t pre[256], lo[256], hi[256];  // per midpoint: first piece, suffix
    uint32_t red[NW + 1];
    unsigned long long red64[NW];
    uint32_t item, full;
};

template <int S>
__device__ inline uint32_t hslot(uint32_t w) {
    constexpr int LOG = __builtin_ctz(S);
    return (w * 0x9E3779B1u) >> (32 - LOG);
}

// Probe step of w (double hashing): odd, so that the S probes of a key
// visit every slot of the power-of-two table once.  Double hashing keeps
// the longest probe sequence of a wave's entries (which the wave waits for)
// shorter than linear probing's clusters do.
template <int S>
__device__ inline uint32_t hstep(uint32_t w) {
    constexpr int LOG = __builtin_ctz(S);
    return ((w * 0xC2B2AE35u) >> (32 - LOG)) | 1u;
}

// Partition of w among P passes (independent of the slot bits).
__device__ inline uint32_t hpart(uint32_t w, uint32_t P) {
    return (uint32_t)(((uint64_t)(w * 0x85EBCA77u) * P) >> 32);
}

// Add one to C_u[w] for the (up to) sixteen entries of a piece whose bits
// are set in `on`; returns the sum of the counters' previous values, or
// HASH_FULL when the table held no free slot for one of them.  Probing runs
// in rounds: every unresolved entry issues its compare-and-swap in the same
// round (entries without work hit the thread's zero word, which the swap of
// 0 for 0 leaves unchanged), so a round costs one LDS round trip; from the
// second round on, an entry index that no lane of the wave still probes
// issues nothing (the wave runs as many rounds as its longest probe
// sequence, and the kernel is bound by instruction issue).  Then the
// sixteen counter additions go out together.
template <int S>
__device__ inline uint32_t hinsert16(uint32_t *key, uint32_t *cnt, uint32_t *zero,
                                     const uint32_t (&w)[16], uint32_t on) {
    uint32_t h[16];
#pragma unroll
    for (int i = 0; i < 16; i++) h[i] = hslot<S>(w[i]);
    uint32_t pend = on;
    for (int round = 0; pend && round < S; round++) {
        // after the first round only a few entry indices are still probed
        // by some lane of the wave: the others issue nothing
        uint64_t act[16];
#pragma unroll
        for (int i = 0; i < 16; i++)
            act[i] = round == 0 ? ~0ull : __builtin_amdgcn_ballot_w64((pend >> i) & 1u);
        uint32_t prev[16];
#pragma unroll
        for (int i = 0; i < 16; i++) {
            const bool p = (pend >> i) & 1u;
            prev[i] = 0u;
            if (act[i]) prev[i] = atomicCAS(p ? &key[h[i]] : zero, 0u, p ? w[i] + 1u : 0u);
        }
#pragma unroll
        for (int i = 0; i < 16; i++) asm volatile("" : "+v"(prev[i]));
#pragma unroll
        for (int i = 0; i < 16; i++) {
            if (!act[i]) continue;
            const bool p = (pend >> i) & 1u;
            const bool done = prev[i] == 0u || prev[i] == w[i] + 1u;
            pend &= ~((uint32_t)(p && done) << i);
            h[i] = (p && !done) ? ((h[i] + hstep<S>(w[i])) & (uint32_t)(S - 1)) : h[i];
        }
    }
    if (pend) return HASH_FULL;
    uint32_t old[16], sft[16];
#pragma unroll
    for (int i = 0; i < 16; i++) {
        const bool p = (on >> i) & 1u;
        sft[i] = (h[i] & 3u) * 8u;
        old[i] = atomicAdd(p ? &cnt[h[i] >> 2] : zero, p ? 1u << sft[i] : 0u);
    }
#pragma unroll
    for (int i = 0; i < 16; i++) asm volatile("" : "+v"(old[i]));
    uint32_t g = 0;
#pragma unroll
    for (int i = 0; i < 16; i++) g += (old[i] >> sft[i]) & 0xFFu;
    return g;
}

template <int NW, int S>
__device__ inline void hclear(HShared<NW, S> &sh) {
    const uint4 z = make_uint4(0, 0, 0, 0);
    sh.zero[threadIdx.x] = 0u;
    for (int i = threadIdx.x; i < S / 4; i += 64 * NW) ((uint4 *)sh.key)[i] = z;
    for (int i = threadIdx.x; i < S / 16; i += 64 * NW) ((uint4 *)sh.cnt)[i] = z;
}

// Last midpoint j < du whose first piece is at or before piece pi.
__device__ inline uint32_t hsearch(const uint32_t *pre, uint32_t du, uint32_t pi) {
    uint32_t j = 0;
    for (uint32_t st = 1u << (31 - __clz(du)); st; st >>= 1) {
        const uint32_t t = j + st;
        const uint32_t pv = pre[(t <= du ? t : du) - 1];
        j = (t <= du && pv <= pi) ? t : j;
    }
    return j - 1;
}

// Walk of one start (d_u <= 255) by the workgroup: returns this thread's
// part of the start's butterflies; *full (workgroup-uniform) when a pass
// filled the table (the partial sum is then meaningless).
template <int NW, int S>
__device__ unsigned long long hash_walk(const CountArgs &a, HShared<NW, S> &sh, uint32_t rb,
                                        uint32_t du, bool &full) {
    constexpr int NTH = 64 * NW;
    constexpr int SL = (256 + NTH - 1) / NTH;
    constexpr uint32_t CAP = S / 2;
    const uint32_t tid = threadIdx.x;
    // midpoints' suffixes (entries after u, all ranked above u) and pieces
    uint32_t run = 0;
    unsigned long long T = 0;
#pragma unroll
    for (int sl = 0; sl < SL; sl++) {
        const uint32_t j = tid + sl * NTH;
        uint32_t lo = 0, hi = 0;
        if (j < du) {
            const uint32_t k = rb + j;
            lo = a.xA[k] + 1u;
            hi = a.offB[a.adjA[k] + 1];
            if (hi < lo) hi = lo;
        }
        const uint32_t np = hi > lo ? (((hi + 3u) >> 2) - (lo >> 2) + WK - 1) / WK : 0u;
        T += hi - lo;
        uint32_t tot;
        const uint32_t ex = block_excl_scan<NTH>(np, sh.red, &tot);
        if (j < 256) {
            sh.pre[j] = run + ex;
            sh.lo[j] = lo;
            sh.hi[j] = hi;
        }
        run += tot;
    }
    T = block_sum64<NTH>(T, sh.red64);          // ends with a barrier
    const uint32_t NP = run;
    const uint32_t pw = (uint32_t)((T + CAP - 1) / CAP);
    const uint32_t P = a.hash_passes ? a.hash_passes : (pw > 1u ? pw : 1u);
    unsigned long long gain = 0;
    full = false;
    for (uint32_t p = 0; p < P; p++) {
        for (uint32_t r0 = 0; r0 < NP; r0 += NTH) {
            const uint32_t pi = r0 + tid;
            const bool valid = pi < NP;
            const uint32_t j = hsearch(sh.pre, du, valid ? pi : 0u);
            const uint32_t lo = sh.lo[j], hi = sh.hi[j];
            const uint32_t g0 = (lo >> 2) + (pi - sh.pre[j]) * WK;
            const uint32_t base = valid ? g0 << 2 : 0u;
            const uint32_t len = valid ? min(hi, (g0 + WK) << 2) - lo : 0u;
            uint4 q[WK];
            wfetch<WK>(a.adjB, Piece{base, lo, len, INF, j}, q);
            uint32_t w[16], on = 0;
#pragma unroll
            for (int k = 0; k < WK; k++) {
                w[4 * k] = q[k].x;
                w[4 * k + 1] = q[k].y;
                w[4 * k + 2] = q[k].z;
                w[4 * k + 3] = q[k].w;
            }
#pragma unroll
            for (int i = 0; i < 16; i++) {
                const uint32_t pos = base + i;
                on |= (uint32_t)((pos - lo) < len && (P == 1u || hpart(w[i], P) == p)) << i;
            }
            const uint32_t g = hinsert16<S>(sh.key, sh.cnt, &sh.zero[threadIdx.x], w, on);
            if (g == HASH_FULL) sh.full = 1u;
            else gain += g;
        }
        __syncthreads();                        // every insert of the pass is done
        const bool f = sh.full != 0u;
        hclear(sh);
        __syncthreads();
        if (f) {
            full = true;
            if (tid == 0) sh.full = 0u;
            __syncthreads();
            return 0;
        }
    }
    return gain;
}

// `chunk` items per access of the class's queue counter.
template <int NW, int S>
__device__ inline uint32_t group_take(HShared<NW, S> &sh, QueueState *q, uint32_t cls,
                                      uint32_t chunk) {
    __syncthreads();
    if (threadIdx.x == 0) sh.item = atomicAdd(&q->head[cls], chunk);
    __syncthreads();
    return sh.item;
}

template <int NW, int S>
__device__ void exact_hash(const CountArgs &a, const uint32_t *items, uint32_t cls) {
    __shared__ HShared<NW, S> sh;
    constexpr int NTH = 64 * NW;
    hclear(sh);
    if (threadIdx.x == 0) sh.full = 0u;
    const uint32_t n = a.q->n_items[cls];
    const uint32_t chunk = NW == 1 ? 16u : 2u;
    unsigned long long acc = 0;
    for (uint32_t b = group_take(sh, a.q, cls, chunk); b < n;
         b = group_take(sh, a.q, cls, chunk)) {
        const uint32_t e = b + chunk < n ? b + chunk : n;
        for (uint32_t it = b; it < e; it++) {
            const uint32_t u = items[it];
            const uint32_t rb = a.offA[u];
            const uint32_t du = a.offA[u + 1] - rb;
            bool full;
            const unsigned long long s = hash_walk<NW, S>(a, sh, rb, du, full);
            if (full) {
                if (threadIdx.x == 0) a.ovf[atomicAdd(&a.q->ovf_count, 1u)] = u;
                continue;
            }
            if (a.per_start) {
                const unsigned long long t = block_sum64<NTH>(s, sh.red64);
                if (threadIdx.x == 0) a.per_start[u] = t;
            }
            acc += s;
        }
    }
    acc = block_sum64<NTH>(acc, sh.red64);
    finish_launch(a.q, cls, acc, nullptr);
}

__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void k_exact_hash_small(CountArgs a) {
    exact_hash<1, HS_SLOTS>(a, a.items_h1, CLS_HASH1);
}

__global__ __launch_bounds__(256) void k_exact_hash_mid(CountArgs a) {
    exact_hash<4, HM_SLOTS>(a, a.items_h2, CLS_HASH2);
}

// ------------------------------------------------------------------ wide: workgroup per start
// Starts with d_u > 255: a workgroup of 8 waves shares a 64 KiB table of
// 32-bit counters over windows of 2^14 ranks (the segment granularity).  The
// midpoints are split into chunks of 64; wave w takes chunks w, w + 8, ...
// and, like the narrow walk, cuts their sub-runs into 16-entry pieces with a
// wave prefix sum, so a window needs workgroup barriers only at its end.
// Each midpoint's cursor (position, segment) lives in registers (starts of
// few midpoints) or in the workspace at the start's adjacency position;
// windows no suffix touches are skipped, and a midpoint without entries in
// a window costs one load there.  LOCAL keeps each midpoint's sub-run of the
// window to read the final counts back in a second pass.
constexpr int NWAVES = NT / WT;
// register cursors per thread in the wide walks (starts of at most WIDE_RC * NT
// midpoints; local counts hold more state per cursor)
constexpr int WIDE_RC = 2, WIDE_RC_L = 1;
constexpr int TBL_WORDS_L = 1 << 14;   // local counts: 64 KiB table, two workgroups per CU

template <int TW>
struct SharedT {
    uint32_t tbl[TW + NT];              // counters, then one zero word per thread
    uint32_t pre[NWAVES][WT], lo[NWAVES][WT], hi[NWAVES][WT], skip[NWAVES][WT];
    uint32_t esum[NWAVES][WT];          // one window's sums of final counts (< 2^14 * 2^16)
    uint32_t own[NWAVES][WT];           // 1 + chunk midpoint at its first piece of a round
    uint32_t red[NWAVES + 1];
    unsigned long long red64[NWAVES];
    uint32_t item;
};

template <int TW>
__device__ inline void clear_table(SharedT<TW> &sh) {
    const uint4 z = make_uint4(0, 0, 0, 0);
    for (int i = threadIdx.x; i < TW / 4; i += NT) ((uint4 *)sh.tbl)[i] = z;
}


// pass 0: add one to the counters of the piece's entries, return the sum of
// previous values; pass 1: return the sum of the final counters.  HALF: two
// 16-bit counters per word (C_u[w] <= d_u <= 65535), else 32-bit counters.
template <int TW, int HALF, int K = WK>
__device__ inline uint32_t cpiece_walk(SharedT<TW> &sh, int pass, const Piece &pc,
                                       const uint4 *q, uint32_t wb) {
    const uint32_t zw = TW + threadIdx.x;
    const uint32_t m = piece_bits<true, 4 * K>(pc);
    uint32_t v[4 * K];
#pragma unroll
    for (int k = 0; k < K; k++) {
        const uint32_t w[4] = {q[k].x, q[k].y, q[k].z, q[k].w};
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const bool on = (m >> (4 * k + i)) & 1u;
            const uint32_t rel = w[i] - wb;
            if (HALF) {
                const uint32_t word = on ? rel >> 1 : zw;
                const uint32_t sft = (rel & 1u) << 4;
                const uint32_t x = pass == 0 ? atomicAdd(&sh.tbl[word], (uint32_t)on << sft)
                                             : sh.tbl[word];
                v[4 * k + i] = (x >> sft) & 0xFFFFu;
            } else {
                const uint32_t idx = on ? rel : zw;
                v[4 * k + i] = pass == 0 ? atomicAdd(&sh.tbl[idx], (uint32_t)on) : sh.tbl[idx];
            }
        }
    }
    // all the piece's LDS operations in flight before the first result is used
#pragma unroll
    for (int k = 0; k < 4 * K; k++) asm volatile("" : "+v"(v[k]));
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < 4 * K; k++) s += v[k];
    return s;
}

// One chunk of 64 midpoints (this wave): publish the sub-runs, walk pieces
// in rounds of 64.  A round's pieces are mapped to midpoints through the
// wave's owner table (midpoints whose first piece falls in the round, plus
// the one carried over), and the next round's pieces are loaded while this
// round's counters are updated (unrolled twice so the buffers swap without
// copies).
template <int TW, int HALF, int K>
__device__ inline void chunk_walk(const CountArgs &a, SharedT<TW> &sh, int pass, uint32_t lo,
                                  uint32_t hi, uint32_t skip, uint32_t wb,
                                  unsigned long long &sum, unsigned long long &esum_mid) {
    const uint32_t lane = threadIdx.x & (WT - 1), wv = threadIdx.x / WT;
    const uint32_t np = hi > lo ? (((hi + 3) >> 2) - (lo >> 2) + K - 1) / K : 0;
    const uint32_t inc = wave_incl_scan(np);
    const uint32_t NP = wave_last(inc);
    const uint32_t first = inc - np;
    sh.pre[wv][lane] = first;
    sh.lo[wv][lane] = lo;
    sh.hi[wv][lane] = hi;
    sh.skip[wv][lane] = skip;
    if (pass == 1) sh.esum[wv][lane] = 0;
    if (NP == 0) {
        esum_mid = 0;
        wave_sync();
        return;
    }
    const uint32_t rounds = (NP + WT - 1) / WT;
    uint32_t carry = 0;
    auto map_round = [&](uint32_t r) -> Piece {
        const uint32_t r0 = r * WT;
        sh.own[wv][lane] = 0;
        wave_sync();
        if (np && first - r0 < (uint32_t)WT) sh.own[wv][first - r0] = lane + 1;
        wave_sync();
        const uint32_t o = max(wave_incl_max(sh.own[wv][lane]), carry);
        carry = wave_last(o);
        const uint32_t j = min((o ? o : 1u) - 1, (uint32_t)(WT - 1));
        const uint32_t pi = r0 + lane;
        const bool valid = pi < NP;
        Piece pc;
        const uint32_t plo = sh.lo[wv][j], phi = sh.hi[wv][j];
        const uint32_t g0 = (plo >> 2) + (pi - sh.pre[wv][j]) * K;
        const uint32_t end = min(phi, (g0 + K) << 2);
        pc.base = valid ? g0 << 2 : 0;
        pc.lo = plo;
        pc.len = valid ? end - plo : 0;
        pc.skip = sh.skip[wv][j];
        pc.j = j;
        return pc;
    };
    uint32_t part = 0;
    auto work = [&](const Piece &pc, const uint4 *q) {
        const uint32_t s = cpiece_walk<TW, HALF, K>(sh, pass, pc, q, wb);
        if (pass == 0) part += s;
        else if (s) atomicAdd(&sh.esum[wv][pc.j], s);
    };
    Piece p0 = map_round(0);
    uint4 q0[K], q1[K];
    wfetch<K>(a.adjB, p0, q0);
    for (uint32_t r = 0;; r += 2) {
        Piece p1 = map_round(r + 1);
        wfetch<K>(a.adjB, p1, q1);
        work(p0, q0);
        if (r + 1 >= rounds) break;
        p0 = map_round(r + 2);
        wfetch<K>(a.adjB, p0, q0);
        work(p1, q1);
        if (r + 2 >= rounds) break;
    }
    sum += part;
    wave_sync();
    if (pass == 1) esum_mid = sh.esum[wv][lane];
    wave_sync();
}

// A table window covers 2^LOGW consecutive segment windows (2^(G_SHIFT +
// LOGW) ranks); each midpoint's sub-run of a table window is the union of
// its (contiguous) segments there, at most 2^LOGW of them.
// Thread tid walks midpoints tid, tid + NT, ... (wave wv's chunks of 64
// start at wv * 64 + c * NT).  With RC > 0 (a start of at most RC * NT
// midpoints) each thread keeps the cursors of its RC midpoints in registers;
// otherwise they live in the workspace and are loaded and stored back once
// per window.
template <bool LOCAL, int TW, int HALF, int LOGW, int RC = 0, int K = WK>
__device__ unsigned long long walk_wide(const CountArgs &a, SharedT<TW> &sh, uint32_t rb,
                                        uint32_t du, const WideScratch &ws, bool pass2,
                                        uint32_t kw_lo = 0, uint32_t kw_hi = INF) {
    static_assert((HALF ? 2 : 1) * TW == (1 << (G_SHIFT + LOGW)), "table covers one window");
    constexpr int R = RC > 0 ? RC : 1;
    const uint32_t tid = threadIdx.x, lane = tid & (WT - 1), wv = tid / WT;
    unsigned long long sum = 0;
    uint32_t mn = INF;
    // register cursors (RC > 0): position, segment, its window and end, list end
    uint32_t cp[R], cs[R], csw[R], cse[R], cev[R], clo[R], chi[R];
    unsigned long long ces[R];
#pragma unroll
    for (int c = 0; c < R; c++) {
        cp[c] = cs[c] = cse[c] = cev[c] = clo[c] = chi[c] = 0;
        csw[c] = INF;
        ces[c] = 0;
    }
    // first cursor of midpoint j: returns p, s, sw, se, ev
    auto start = [&](uint32_t j, uint32_t &p, uint32_t &s, uint32_t &sw, uint32_t &se,
                     uint32_t &ev) {
        const uint32_t k = rb + j;
        const uint32_t v = a.adjA[k];
        const uint32_t pb = a.offB[v];
        ev = a.offB[v + 1];
        p = LOCAL ? pb : a.xA[k] + 1;
        s = 0;
        sw = INF;
        se = 0;
        // windows [kw_lo, kw_hi) only: the cursor starts at the first entry
        // of window kw_lo or later
        if (kw_lo && p < ev) p = lower_bound_glb(a.adjB, p, ev, kw_lo << (G_SHIFT + LOGW));
        if (LOCAL ? (ev - pb > 1 && p < ev) : (p < ev)) {
            s = a.seg1[p] - 1;
            sw = a.seg_win[s];
            se = a.seg_start[s + 1];
            mn = min(mn, sw >> LOGW);
        } else {
            p = ev;                             // nothing to walk
        }
    };
    // sub-run [lo, hi) of window kw and the cursor moved past it
    auto advance = [&](uint32_t kw, uint32_t &p, uint32_t &s, uint32_t &sw, uint32_t &se,
                       uint32_t ev, uint32_t &lo, uint32_t &hi) {
        lo = hi = 0;
        if (p < ev && (sw >> LOGW) == kw) {
            lo = p;
            uint32_t e = se, nsw = INF, nse = 0;
            s++;
            if (e < ev) {
                nsw = a.seg_win[s];
                nse = a.seg_start[s + 1];
            }
            while (e < ev && (nsw >> LOGW) == kw) {
                e = nse;
                s++;
                if (e < ev) {
                    nsw = a.seg_win[s];
                    nse = a.seg_start[s + 1];
                }
            }
            hi = e < ev ? e : ev;
            p = hi;
            sw = p < ev ? nsw : INF;
            se = nse;
        }
    };
    if (RC > 0) {
#pragma unroll
        for (int c = 0; c < R; c++) {
            const uint32_t j = tid + c * NT;
            if (j < du) start(j, cp[c], cs[c], csw[c], cse[c], cev[c]);
        }
    }
    // workspace cursors: a start whose remaining entries are fewer than its
    // (midpoint, window) pairs ("lazy") loads a cursor's other fields only
    // when its segment window is the current one; a dense start loads them
    // all in one round
    bool lazy = false;
    if (RC == 0) {
        unsigned long long rem = 0;
        for (uint32_t j = tid; j < du; j += NT) {
            const uint64_t x = ws.at(j, rb + j);
            uint32_t p, s, sw, se, ev;
            start(j, p, s, sw, se, ev);
            rem += ev - p;
            ws.pos[x] = p;
            ws.seg[x] = s;
            ws.lim[x] = ev;
            ws.sw[x] = sw;
            ws.se[x] = se;
            if (LOCAL) {
                ws.lo[x] = ws.hi[x] = 0;
                ws.esum[x] = 0;
            }
        }
        rem = block_sum64<NT>(rem, sh.red64);
        const uint64_t nwin = ((uint64_t)(a.nA - 1) >> (G_SHIFT + LOGW)) + 1;
        lazy = rem < (uint64_t)du * (nwin - (kw_lo < nwin ? kw_lo : 0));
    }
    uint32_t kw = block_min<NT>(mn, sh.red);
    while (kw < kw_hi) {                        // INF >= kw_hi: no window left
        const uint32_t wb = kw << (G_SHIFT + LOGW);
        uint32_t next = INF;
        if (RC > 0) {
#pragma unroll
            for (int c = 0; c < R; c++) {
                if (wv * WT + c * NT >= du) break;      // wave-uniform
                const uint32_t j = tid + c * NT;
                uint32_t lo = 0, hi = 0, skip = INF;
                if (j < du) {
                    advance(kw, cp[c], cs[c], csw[c], cse[c], cev[c], lo, hi);
                    if (cp[c] < cev[c]) next = min(next, csw[c] >> LOGW);
                    if (LOCAL) {
                        skip = a.xA[rb + j];
                        clo[c] = lo;
                        chi[c] = hi;
                    }
                }
                unsigned long long unused;
                chunk_walk<TW, HALF, K>(a, sh, 0, lo, hi, skip, wb, sum, unused);
            }
        } else {
            for (uint32_t cb = wv * WT; cb < du; cb += NT) {
                const uint32_t j = cb + lane, k = rb + j;
                const uint64_t x = ws.at(j, k);
                uint32_t lo = 0, hi = 0, skip = INF;
                if (j < du) {
                    // lazy: a midpoint without entries in this window costs
                    // one load (its segment window; INF once its list is
                    // done); else the cursor in one round of independent loads
                    uint32_t ev = 0, p = 0, s = 0, se = 0;
                    if (!lazy) {
                        ev = ws.lim[x];
                        p = ws.pos[x];
                        s = ws.seg[x];
                        se = ws.se[x];
                    }
                    uint32_t sw = ws.sw[x];
                    if ((sw >> LOGW) == kw) {
                        if (lazy) {
                            ev = ws.lim[x];
                            p = ws.pos[x];
                            s = ws.seg[x];
                            se = ws.se[x];
                        }
                        advance(kw, p, s, sw, se, ev, lo, hi);
                        ws.pos[x] = p;
                        ws.seg[x] = s;
                        ws.sw[x] = sw;
                        ws.se[x] = se;
                        if (LOCAL) skip = a.xA[k];
                    }
                    // the window's sub-run for the second look (lazy: only
                    // a nonempty one, which the second look empties again)
                    if (LOCAL && (!lazy || hi > lo)) {
                        ws.lo[x] = lo;
                        ws.hi[x] = hi;
                    }
                    if (sw != INF) next = min(next, sw >> LOGW);     // INF: list done
                }
                unsigned long long unused;
                chunk_walk<TW, HALF, K>(a, sh, 0, lo, hi, skip, wb, sum, unused);
            }
        }
        if (LOCAL && pass2) {
            __syncthreads();                    // all counts of the window are final
            if (RC > 0) {
#pragma unroll
                for (int c = 0; c < R; c++) {
                    if (wv * WT + c * NT >= du) break;
                    const uint32_t j = tid + c * NT;
                    const bool in = j < du;
                    unsigned long long e = 0;
                    chunk_walk<TW, HALF, K>(a, sh, 1, in ? clo[c] : 0u, in ? chi[c] : 0u,
                                         in ? a.xA[rb + j] : INF, wb, sum, e);
                    ces[c] += in ? e : 0ull;
                }
            } else {
                for (uint32_t cb = wv * WT; cb < du; cb += NT) {
                    const uint32_t j = cb + lane, k = rb + j;
                    const uint64_t x = ws.at(j, k);
                    uint32_t lo = 0, hi = 0, skip = INF;
                    if (j < du) {
                        lo = ws.lo[x];
                        hi = ws.hi[x];
                        if (hi > lo) {
                            skip = a.xA[k];
                            if (lazy) ws.hi[x] = lo;
                        }
                    }
                    unsigned long long e = 0;
                    chunk_walk<TW, HALF, K>(a, sh, 1, lo, hi, skip, wb, sum, e);
                    if (j < du && e) ws.esum[x] += e;
                }
            }
        }
        __syncthreads();
        clear_table(sh);
        kw = block_min<NT>(next, sh.red);
    }
    if (LOCAL && RC > 0) {
#pragma unroll
        for (int c = 0; c < R; c++) {
            const uint32_t j = tid + c * NT;
            if (j < du) ws.esum[ws.at(j, rb + j)] = ces[c];
        }
    }
    return sum;
}

// A wide start whose wedges (below 2^b, b the plan's bucket) are at most its
// (midpoint, table window) pairs over the windows it walks (from rank lo)
// has sub-runs of about one entry: its pieces are WK_WIDE_SPARSE groups.
constexpr int WK_WIDE_SPARSE = 1;
__device__ inline bool wide_sparse(uint16_t bucket, uint32_t du, uint32_t nA, uint32_t lo) {
    const uint32_t b = bucket & 255u, logw = du <= 0xFFFFu ? 1u : 0u;
    const uint64_t nwin = ((uint64_t)(nA - 1) >> (G_SHIFT + logw)) + 1 - (lo >> (G_SHIFT + logw));
    return b < 63 && (1ull << b) <= (uint64_t)du * nwin;
}

template <int TW>
__device__ inline uint32_t block_take(SharedT<TW> &sh, QueueState *q) {
    __syncthreads();
    if (threadIdx.x == 0) sh.item = atomicAdd(&q->head[1], 1u);
    __syncthreads();
    return sh.item;
}

__global__ __launch_bounds__(NT) void k_exact_wide(CountArgs a, WideScratch ws) {
    __shared__ SharedT<TBL_WORDS> sh;
    clear_table(sh);
    sh.tbl[TBL_WORDS + threadIdx.x] = 0;
    const uint32_t n = a.q->n_items[1];
    unsigned long long acc = 0;
    for (uint32_t it = block_take(sh, a.q); it < n; it = block_take(sh, a.q)) {
        const uint32_t u = a.items_wide[it];
        const uint32_t rb = a.offA[u];
        const uint32_t du = a.offA[u + 1] - rb;
        // 16-bit counters over two segment windows when C_u[w] <= d_u fits
        const bool sp = wide_sparse(a.bucket[u], du, a.nA, u);
        const unsigned long long s =
            du <= WIDE_RC * NT
                ? (sp ? walk_wide<false, TBL_WORDS, 1, 1, WIDE_RC, WK_WIDE_SPARSE>(a, sh, rb, du, ws,
                                                                                   false)
                      : walk_wide<false, TBL_WORDS, 1, 1, WIDE_RC>(a, sh, rb, du, ws, false))
            : du <= 0xFFFFu
                ? (sp ? walk_wide<false, TBL_WORDS, 1, 1, 0, WK_WIDE_SPARSE>(a, sh, rb, du, ws, false)
                      : walk_wide<false, TBL_WORDS, 1, 1>(a, sh, rb, du, ws, false))
                : walk_wide<false, TBL_WORDS, 0, 0>(a, sh, rb, du, ws, false);
        if (a.per_start) {
            const unsigned long long t = block_sum64<NT>(s, sh.red64);
            if (threadIdx.x == 0) a.per_start[u] = t;
        }
        acc += s;
    }
    acc = block_sum64<NT>(acc, sh.red64);
    finish_launch(a.q, 1, acc, a.total);
}

// Local counts of wide starts: 16-bit counters over windows of 2^15 ranks
// when d_u <= 65535 (two segment windows per table), else 32-bit counters
// over 2^14.
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_local_wide(LocalArgs a,
                                                                                   WideScratch ws) {
    __shared__ SharedT<TBL_WORDS_L> sh;
    __shared__ uint32_t last;
    clear_table(sh);
    sh.tbl[TBL_WORDS_L + threadIdx.x] = 0;
    const uint32_t n = a.c.q->n_items[CLS_WIDE];
    const uint32_t tid = threadIdx.x;
    for (uint32_t it = block_take(sh, a.c.q); it < n; it = block_take(sh, a.c.q)) {
        const uint32_t u = a.c.items_wide[it];
        const uint32_t gG = a.wide_g[it], g = gG & 0xFFFFu, G = gG >> 16;
        const uint32_t rb = a.c.offA[u], du = a.c.offA[u + 1] - rb;
        const uint32_t logw = du <= 0xFFFFu ? 1u : 0u;
        const uint32_t nwin = ((a.c.nA - 1) >> (G_SHIFT + logw)) + 1;
        const uint32_t kw_lo = (uint32_t)((uint64_t)g * nwin / G);
        const uint32_t kw_hi = g + 1 == G ? INF : (uint32_t)((uint64_t)(g + 1) * nwin / G);
        const bool sp = wide_sparse(a.c.bucket[u], du, a.c.nA, 0);
        unsigned long long s =
            du <= WIDE_RC_L * NT
                ? (sp ? walk_wide<true, TBL_WORDS_L, 1, 1, WIDE_RC_L, WK_WIDE_SPARSE>(
                            a.c, sh, rb, du, ws, a.pass2, kw_lo, kw_hi)
                      : walk_wide<true, TBL_WORDS_L, 1, 1, WIDE_RC_L>(a.c, sh, rb, du, ws, a.pass2,
                                                                      kw_lo, kw_hi))
            : du <= 0xFFFFu
                ? (sp ? walk_wide<true, TBL_WORDS_L, 1, 1, 0, WK_WIDE_SPARSE>(a.c, sh, rb, du, ws,
                                                                             a.pass2, kw_lo, kw_hi)
                      : walk_wide<true, TBL_WORDS_L, 1, 1>(a.c, sh, rb, du, ws, a.pass2, kw_lo,
                                                           kw_hi))
                : walk_wide<true, TBL_WORDS_L, 0, 0>(a.c, sh, rb, du, ws, a.pass2, kw_lo, kw_hi);
        __syncthreads();
        s = block_sum64<NT>(s, sh.red64);
        if (G == 1) {
            if (a.pass2) {
                for (uint32_t j = tid; j < du; j += NT) {
                    const uint32_t k = rb + j;
                    const uint32_t v = a.c.adjA[k];
                    emit_edge(a, k, v, a.c.offB[v + 1] - a.c.offB[v], ws.esum[ws.at(j, k)]);
                }
            }
            if (tid == 0 && a.cntA) a.cntA[a.idA[u]] = s;
            continue;
        }
        // one part of a split start
        if (a.pass2) {
            for (uint32_t j = tid; j < du; j += NT) {
                const unsigned long long e = ws.esum[ws.at(j, rb + j)];
                if (e) atomicAdd(&a.esum_g[rb + j], e);
            }
        }
        if (tid == 0 && a.cntA && s) atomicAdd(&a.cntA[a.idA[u]], s);
        __syncthreads();
        if (tid == 0) {
            __threadfence();
            last = atomicAdd(&a.wdone[u], 1u) == G - 1;
        }
        __syncthreads();
        if (last && a.pass2) {
            __threadfence();
            for (uint32_t j = tid; j < du; j += NT) {
                const uint32_t k = rb + j;
                const uint32_t v = a.c.adjA[k];
                emit_edge(a, k, v, a.c.offB[v + 1] - a.c.offB[v], atomicAdd(&a.esum_g[k], 0ull));
            }
        }
    }
    finish_launch(a.c.q, CLS_WIDE, 0, nullptr);
}

// Per-part totals of a disjoint union counted from L: part q owns the L ids
// [part_l[q], part_l[q + 1]); its total is the sum of its starts' counts,
// added in a fixed order (strided per thread, then the block reduction).
// rank_l == NULL: the ids are the ranks.
__global__ __launch_bounds__(256) void k_part_sums(const unsigned long long *per_start,
                                                   const uint32_t *rank_l, const uint32_t *part_l,
                                                   uint32_t nparts, unsigned long long *totals) {
    __shared__ unsigned long long red[256 / WAVE];
    for (uint32_t q = blockIdx.x; q < nparts; q += gridDim.x) {
        unsigned long long t = 0;
        for (uint32_t id = part_l[q] + threadIdx.x; id < part_l[q + 1]; id += blockDim.x)
            t += per_start[rank_l ? rank_l[id] : id];
        t = block_sum64<256>(t, red);
        if (threadIdx.x == 0) totals[q] = t;
    }
}

// B_v of the midpoint side: half the sum of its edges' counts (each
// butterfly through v uses two edges of v), read through the B-side row's
// cross positions; one wave per row, outputs in caller ids.
__global__ __launch_bounds__(256) void k_local_finish(const uint32_t *offB, const uint32_t *xB,
                                                      const unsigned long long *epos,
                                                      const uint32_t *idB, uint32_t nB,
                                                      unsigned long long *cntB) {
    const uint32_t lane = threadIdx.x & (WAVE - 1), wpb = blockDim.x / WAVE;
    for (uint32_t v = blockIdx.x * wpb + threadIdx.x / WAVE; v < nB; v += gridDim.x * wpb) {
        unsigned long long t = 0;
        for (uint32_t p = offB[v] + lane; p < offB[v + 1]; p += WAVE) t += epos[xB[p]];
        t = wave_sum64(t);
        if (lane == 0) cntB[idB[v]] = t >> 1;
    }
}

// ------------------------------------------------------------------ host side
struct ExactWs {
    uint32_t *seg1, *seg_start, *seg_win, *scan_tmp, *items, *items_wide, *items_h1, *items_h2;
    uint32_t *ovf, *wide_g, *wdone;
    uint32_t *wpos, *wseg, *wlim, *wsw, *wse;
    uint16_t *bucket, *nsplit;
    QueueState *q;
};

// Items of the wide class: one per start, plus the extra parts of split
// starts: at most 2 * wedges / split in all (every start's all-ends wedges
// add up to twice the wedges), and at most one per further table window.
static inline size_t wide_items_cap(const Plan &p) {
    if (!p.split) return pad64(p.nA) + 64;
    // extra parts: at most all-ends wedges / split, and at most one per
    // further table window of every start
    const uint64_t by_wedges = 2 * (p.wedges / p.split);
    const uint64_t by_windows = (uint64_t)p.nA * (p.nA ? ((p.nA - 1) >> G_SHIFT) : 0);
    return pad64(p.nA) + (size_t)(by_wedges < by_windows ? by_wedges : by_windows) + 64;
}

static ExactWs carve_exact(Carver &c, const Plan &p) {
    ExactWs w;
    w.seg1 = c.take<uint32_t>(pad64(p.m));
    w.seg_start = c.take<uint32_t>(pad64(p.m + 3));   // look-ahead reads up to segments + 2
    w.seg_win = c.take<uint32_t>(pad64(p.m + 2));
    w.scan_tmp = c.take<uint32_t>(scan_tmp_elems(p.m));
    w.items = c.take<uint32_t>(pad64(p.nA));
    w.items_wide = c.take<uint32_t>(wide_items_cap(p));
    w.wide_g = c.take<uint32_t>(wide_items_cap(p));
    w.wdone = c.take<uint32_t>(pad64(p.nA));
    w.nsplit = c.take<uint16_t>(pad64(p.nA));
    w.items_h1 = c.take<uint32_t>(pad64(p.nA));
    w.items_h2 = c.take<uint32_t>(pad64(p.nA));
    w.ovf = c.take<uint32_t>(pad64(p.nA));
    w.wpos = c.take<uint32_t>(pad64(p.m));
    w.wseg = c.take<uint32_t>(pad64(p.m));
    w.wlim = c.take<uint32_t>(pad64(p.m));
    w.wsw = c.take<uint32_t>(pad64(p.m));
    w.wse = c.take<uint32_t>(pad64(p.m));
    w.bucket = c.take<uint16_t>(pad64(p.nA));
    w.q = c.take<QueueState>(1);
    return w;
}

static inline unsigned grid_for(uint64_t n, int nt = 256) {
    uint64_t g = (n + nt - 1) / nt;
    if (g < 1) g = 1;
    if (g > 65535ull * 16) g = 65535ull * 16;
    return (unsigned)g;
}

// Upper bound of the count: every start's pairs gain at most (d_u - 1) per
// wedge / 2, so B <= wedges * (max start degree - 1) / 2.
static bool overflow_risk(uint64_t wedges, uint32_t max_deg) {
    if (max_deg < 2) return false;
    unsigned __int128 b = (unsigned __int128)wedges * (max_deg - 1) / 2;
    return b >> 64;
}

// Segments, per-start work buckets and the work queues for one plan.
// Wedge limits of the two hash classes (0: none; the local counts use none).
struct HashLimits {
    uint32_t small, mid, density;
};
constexpr HashLimits HASH_DEFAULT = {HS_DEFAULT, HM_MAX, HASH_DENSITY}, HASH_NONE = {0, 0, 0};

static int prepare(const Plan &p, ExactWs &w, int all_ends, const uint8_t *mark, hipStream_t s,
                   uint32_t narrow_max = NARROW_MAX, HashLimits hl = HASH_NONE,
                   uint64_t split = 0) {
    k_zero_u32<<<1, 256, 0, s>>>((uint32_t *)w.q, (uint64_t)(sizeof(QueueState) / 4));
    if (p.m) {
        k_seg_flags<<<grid_for(p.m), 256, 0, s>>>(p.adjB, p.m, w.seg1);
        k_seg_rowstarts<<<grid_for(p.nB), 256, 0, s>>>(p.offB, p.nB, w.seg1);
        BFC_HIP(hipGetLastError());
        BFC_TRY(scan_u32_inclusive(w.seg1, w.seg1, p.m, w.scan_tmp, s));
        k_seg_fill<<<grid_for(p.m), 256, 0, s>>>(p.adjB, p.m, w.seg1, w.seg_start, w.seg_win);
        BFC_HIP(hipGetLastError());
    }
    if (p.nA) {
        unsigned g = grid_for(p.nA, 4);
        if (g > 8192) g = 8192;
        k_work<<<g, 256, 0, s>>>(p.offA, p.adjA, p.xA, p.offB, p.adjB, p.nA, all_ends, mark,
                                 narrow_max,
                                 hl.small, hl.mid, hl.density, HALF_DENSITY, split, w.bucket,
                                 split ? w.nsplit : nullptr,
                                 w.q);
        BFC_HIP(hipGetLastError());
    }
    k_bucket_offsets<<<1, 64, 0, s>>>(w.q);
    if (p.nA)
        k_scatter_items<<<grid_for(p.nA), 256, 0, s>>>(
            w.bucket, p.nA, w.q, ItemLists{{w.items, w.items_wide, w.items_h1, w.items_h2},
                                           w.wide_g, split ? w.nsplit : nullptr});
    BFC_HIP(hipGetLastError());
    return BFC_OK;
}

static void fill_args(const Plan &p, const ExactWs &w, CountArgs &a) {
    a.offA = p.offA; a.adjA = p.adjA; a.xA = p.xA; a.offB = p.offB; a.adjB = p.adjB;
    a.seg1 = w.seg1; a.seg_start = w.seg_start; a.seg_win = w.seg_win;
    a.items = w.items; a.items_wide = w.items_wide; a.items_h1 = w.items_h1;
    a.items_h2 = w.items_h2; a.ovf = w.ovf; a.q = w.q; a.nA = p.nA; a.total = nullptr;
    a.bucket = w.bucket;
    a.chunk = WCHUNK; a.per_start = nullptr; a.hash_passes = 0;
}

// Tuning with defaults filled in and ranges checked.
static int resolve_tuning(const bfc_tuning *t, bfc_tuning &r) {
    r.narrow_max = NARROW_MAX;
    r.chunk = WCHUNK;
    r.narrow_waves_per_cu = 8;
    r.wide_groups_per_cu = 2;
    r.hash_small_max = HS_DEFAULT;
    r.hash_mid_max = HM_MAX;
    r.hash_passes = 0;
    r.hash_max_density = HASH_DENSITY;
    if (!t) return BFC_OK;
    r.hash_passes = t->hash_passes;
    if (t->hash_max_density) r.hash_max_density = t->hash_max_density;
    if (t->narrow_max) r.narrow_max = t->narrow_max;
    if (t->chunk) r.chunk = t->chunk;
    if (t->narrow_waves_per_cu) r.narrow_waves_per_cu = t->narrow_waves_per_cu;
    if (t->wide_groups_per_cu) r.wide_groups_per_cu = t->wide_groups_per_cu;
    if (t->hash_small_max) r.hash_small_max = t->hash_small_max == BFC_HASH_OFF ? 0 : t->hash_small_max;
    if (t->hash_mid_max) r.hash_mid_max = t->hash_mid_max == BFC_HASH_OFF ? 0 : t->hash_mid_max;
    if (r.narrow_max > NARROW_MAX || r.chunk > 64 || r.narrow_waves_per_cu > 8 ||
        r.wide_groups_per_cu > 2 || r.hash_small_max > HS_MAX || r.hash_mid_max > HM_MAX ||
        r.hash_passes > HASH_PASSES)
        return BFC_E_ARG;
    return BFC_OK;
}

static HashLimits hash_limits(const bfc_tuning &r) {
    return HashLimits{r.hash_small_max, r.hash_mid_max, r.hash_max_density};
}

// Waves of the narrow grid per CU (LDS bound: eight 16 KiB tables) and
// workgroups of the wide grid (two 64 KiB tables).
static int grids(unsigned &narrow, unsigned &wide, const bfc_tuning *t = nullptr,
                 unsigned *hsmall = nullptr, unsigned *hmid = nullptr) {
    bfc_tuning r;
    BFC_TRY(resolve_tuning(t, r));
    int dev = 0;
    BFC_HIP(hipGetDevice(&dev));
    const unsigned cu = (unsigned)device_cu_count(dev);
    narrow = cu * r.narrow_waves_per_cu;
    wide = cu * r.wide_groups_per_cu;
    // hash kernels: 8.2 KiB of LDS per one-wave group, 44 KiB per mid group
    if (hsmall) *hsmall = cu * 16;
    if (hmid) *hmid = cu * 3;
    return BFC_OK;
}

static int exact_setup(const bfc_graph *g, int side, void *d_ws, size_t ws_bytes, Plan &p,
                       ExactWs &w) {
    if (!d_ws) return BFC_E_NULL;
    BFC_TRY(make_plan(g, side, &p));
    if (!aligned256(d_ws)) return BFC_E_ALIGN;
    if (overflow_risk(p.wedges, p.max_deg_A)) return BFC_E_OVERFLOW_RISK;
    Carver c(d_ws, ws_bytes);
    w = carve_exact(c, p);
    if (!c.fits()) return BFC_E_WS_SMALL;
    return BFC_OK;
}

// Local counts: the exact count's workspace, the midpoint sums, the edge
// sums of split starts, and each wide workgroup's slice of cursor state.
struct LocalWs {
    ExactWs e;
    unsigned long long *epos, *esum_g;
    WideScratch slices;
};

static LocalWs carve_local(Carver &c, const Plan &p, unsigned wide_groups) {
    LocalWs w;
    w.e = carve_exact(c, p);
    w.epos = c.take<unsigned long long>(pad64(p.m));
    w.esum_g = c.take<unsigned long long>(pad64(p.m));
    const uint64_t stride = pad64(p.max_deg_A);
    const uint64_t n = (uint64_t)wide_groups * stride;
    WideScratch &x = w.slices;
    x.pos = c.take<uint32_t>(n);
    x.seg = c.take<uint32_t>(n);
    x.lim = c.take<uint32_t>(n);
    x.sw = c.take<uint32_t>(n);
    x.se = c.take<uint32_t>(n);
    x.lo = c.take<uint32_t>(n);
    x.hi = c.take<uint32_t>(n);
    x.esum = c.take<unsigned long long>(n);
    x.stride = stride;
    return w;
}

// Workgroups of the local counts' wide grid (default launch shape).
static int local_wide_groups(unsigned &gw) {
    unsigned gn;
    return grids(gn, gw);
}

// Workspace of bfc_exact for any graph with these sizes (either side).
size_t exact_ws_bound(uint32_t nl, uint32_t nr, uint64_t m) {
    Plan p = {};
    p.nA = nl > nr ? nl : nr;
    p.nB = p.nA;
    p.m = m;
    Carver c(nullptr, 0);
    carve_exact(c, p);
    return c.used;
}

int local_ws_size(const bfc_graph *g, int side, size_t *bytes, uint64_t split) {
    if (!bytes) return BFC_E_NULL;
    Plan p;
    BFC_TRY(make_plan(g, side, &p));
    p.split = split ? split : SPLIT_WEDGES;
    unsigned gw;
    BFC_TRY(local_wide_groups(gw));
    Carver c(nullptr, 0);
    carve_local(c, p, gw);
    *bytes = c.used;
    return BFC_OK;
}

// Local counts of the starts on `side` (all, or those whose mark[rank] is
// set), written into caller-zeroed outputs: B_u of the starts (caller ids),
// and when asked, B_e of their edges (caller order) and B_v of the midpoints
// (from the processed starts' edges only).
int local_run(const bfc_graph *g, int side, const uint8_t *mark, uint64_t *d_cnt_l,
              uint64_t *d_cnt_r, uint64_t *d_cnt_e, void *d_ws, size_t ws_bytes,
              hipStream_t s, uint64_t split) {
    if (!d_ws || (!d_cnt_l && !d_cnt_r && !d_cnt_e)) return BFC_E_NULL;
    Plan p;
    BFC_TRY(make_plan(g, side, &p));
    p.split = split ? split : SPLIT_WEDGES;
    if (!aligned256(d_ws)) return BFC_E_ALIGN;
    if (p.wedges >> 63 || overflow_risk(2 * p.wedges, p.max_deg_A)) return BFC_E_OVERFLOW_RISK;
    unsigned gn, gw;
    BFC_TRY(grids(gn, gw));
    Carver c(d_ws, ws_bytes);
    LocalWs w = carve_local(c, p, gw);
    if (!c.fits()) return BFC_E_WS_SMALL;
    unsigned long long *cl = (unsigned long long *)d_cnt_l, *cr = (unsigned long long *)d_cnt_r,
                       *ce = (unsigned long long *)d_cnt_e;
    unsigned long long *cntB = p.start_r ? cl : cr;
    const bool pass2 = ce != nullptr || cntB != nullptr;
    if (cntB) k_zero_u64<<<grid_for(p.m), 256, 0, s>>>(w.epos, p.m);
    k_zero_u32<<<grid_for(p.nA), 256, 0, s>>>(w.e.wdone, p.nA);
    if (pass2) k_zero_u64<<<grid_for(p.m), 256, 0, s>>>(w.esum_g, p.m);
    BFC_HIP(hipGetLastError());
    BFC_TRY(prepare(p, w.e, 1, mark, s, NARROW_MAX, HASH_NONE, p.split));
    if (p.nA == 0 || p.m == 0) return BFC_OK;
    LocalArgs a;
    fill_args(p, w.e, a.c);
    a.eidA = p.start_r ? g->eid_r : g->eid_l;
    a.idA = p.start_r ? g->id_r : g->id_l;
    a.cntA = p.start_r ? cr : cl;
    a.cntE = ce;
    a.epos = cntB ? w.epos : nullptr;
    a.pass2 = pass2;
    a.wide_g = w.e.wide_g;
    a.wdone = w.e.wdone;
    a.esum_g = w.esum_g;
    k_local_narrow<<<gn, WT, 0, s>>>(a);
    k_local_wide<<<gw, NT, 0, s>>>(a, w.slices);
    if (cntB)
        k_local_finish<<<grid_for(p.nB, 4) < 8192 ? grid_for(p.nB, 4) : 8192, 256, 0, s>>>(
            p.offB, p.start_r ? g->xpos_l : g->xpos_r, w.epos, p.start_r ? g->id_l : g->id_r,
            p.nB, cntB);
    BFC_HIP(hipGetLastError());
    return BFC_OK;
}

// The two persistent launches of one count on a planned workspace.
static int launch_count(const Plan &p, const ExactWs &w, const bfc_tuning *t,
                        unsigned long long *total, unsigned long long *per_start, hipStream_t s) {
    if (p.nA == 0 || p.m == 0) {
        k_zero_u64<<<1, 64, 0, s>>>(total, 1);
        BFC_HIP(hipGetLastError());
        return BFC_OK;
    }
    bfc_tuning r;
    BFC_TRY(resolve_tuning(t, r));
    CountArgs a;
    fill_args(p, w, a);
    a.chunk = r.chunk;
    a.hash_passes = r.hash_passes;
    a.per_start = per_start;
    unsigned gn, gw, ghs, ghm;
    BFC_TRY(grids(gn, gw, &r, &ghs, &ghm));
    // hash starts first: a start they give back is walked by the narrow launch
    k_exact_hash_small<<<ghs, 64, 0, s>>>(a);
    k_exact_hash_mid<<<ghm, 256, 0, s>>>(a);
    k_exact_narrow<<<gn, WT, 0, s>>>(a);
    a.total = total;
    WideScratch ws = {w.wpos, w.wseg, w.wlim, w.wsw, w.wse, nullptr, nullptr, nullptr, 0};
    k_exact_wide<<<gw, NT, 0, s>>>(a, ws);
    BFC_HIP(hipGetLastError());
    return BFC_OK;
}

}  // namespace bfc

using namespace bfc;

extern "C" {

int bfc_side_used(const bfc_graph *g, int side) {
    Plan p;
    BFC_TRY(make_plan(g, side, &p));
    return p.start_r ? BFC_SIDE_R : BFC_SIDE_L;
}

int bfc_wedges(const bfc_graph *g, int side, uint64_t *wedges) {
    if (!wedges) return BFC_E_NULL;
    Plan p;
    BFC_TRY(make_plan(g, side, &p));
    *wedges = p.wedges;
    return BFC_OK;
}

int bfc_exact_ws_size(const bfc_graph *g, int side, size_t *bytes) {
    if (!bytes) return BFC_E_NULL;
    Plan p;
    BFC_TRY(make_plan(g, side, &p));
    Carver c(nullptr, 0);
    carve_exact(c, p);
    *bytes = c.used;
    return BFC_OK;
}

int bfc_exact_plan(const bfc_graph *g, int side, void *d_ws, size_t ws_bytes, hipStream_t s) {
    Plan p;
    ExactWs w;
    BFC_TRY(exact_setup(g, side, d_ws, ws_bytes, p, w));
    return prepare(p, w, 0, nullptr, s, NARROW_MAX, HASH_DEFAULT);
}

int bfc_exact_count(const bfc_graph *g, int side, uint64_t *d_total, void *d_ws,
                    size_t ws_bytes, hipStream_t s) {
    if (!d_total) return BFC_E_NULL;
    if ((uintptr_t)d_total & 7) return BFC_E_ALIGN;
    Plan p;
    ExactWs w;
    BFC_TRY(exact_setup(g, side, d_ws, ws_bytes, p, w));
    return launch_count(p, w, nullptr, (unsigned long long *)d_total, nullptr, s);
}

int bfc_exact(const bfc_graph *g, int side, uint64_t *d_total, void *d_ws, size_t ws_bytes,
              hipStream_t s) {
    if (!d_total) return BFC_E_NULL;
    BFC_TRY(bfc_exact_plan(g, side, d_ws, ws_bytes, s));
    return bfc_exact_count(g, side, d_total, d_ws, ws_bytes, s);
}

int bfc_exact_tuned(const bfc_graph *g, int side, const bfc_tuning *t, uint64_t *d_total,
                    void *d_ws, size_t ws_bytes, hipStream_t s) {
    if (!d_total) return BFC_E_NULL;
    if ((uintptr_t)d_total & 7) return BFC_E_ALIGN;
    bfc_tuning r;
    BFC_TRY(resolve_tuning(t, r));
    Plan p;
    ExactWs w;
    BFC_TRY(exact_setup(g, side, d_ws, ws_bytes, p, w));
    BFC_TRY(prepare(p, w, 0, nullptr, s, r.narrow_max, hash_limits(r)));
    return launch_count(p, w, &r, (unsigned long long *)d_total, nullptr, s);
}

int bfc_exact_parts_ws_size(const bfc_graph *g, size_t *bytes) {
    if (!bytes) return BFC_E_NULL;
    Plan p;
    BFC_TRY(make_plan(g, BFC_SIDE_L, &p));
    Carver c(nullptr, 0);
    carve_exact(c, p);
    c.take<unsigned long long>(pad64(p.nA));
    c.take<unsigned long long>(1);
    *bytes = c.used;
    return BFC_OK;
}

int bfc_exact_parts(const bfc_graph *g, uint32_t nparts, const uint32_t *d_part_l,
                    const bfc_tuning *t, uint64_t *d_totals, void *d_ws, size_t ws_bytes,
                    hipStream_t s) {
    if (!g || !d_part_l || !d_totals || !d_ws) return BFC_E_NULL;
    if (nparts == 0) return BFC_E_ARG;
    if ((uintptr_t)d_totals & 7) return BFC_E_ALIGN;
    bfc_tuning r;
    BFC_TRY(resolve_tuning(t, r));
    Plan p;
    ExactWs w;
    BFC_TRY(exact_setup(g, BFC_SIDE_L, d_ws, ws_bytes, p, w));
    Carver c(d_ws, ws_bytes);
    carve_exact(c, p);
    unsigned long long *per_start = c.take<unsigned long long>(pad64(p.nA));
    unsigned long long *total = c.take<unsigned long long>(1);
    if (!c.fits()) return BFC_E_WS_SMALL;
    k_zero_u64<<<grid_for(p.nA), 256, 0, s>>>(per_start, p.nA);
    BFC_HIP(hipGetLastError());
    BFC_TRY(prepare(p, w, 0, nullptr, s, r.narrow_max, hash_limits(r)));
    BFC_TRY(launch_count(p, w, &r, total, per_start, s));
    unsigned gp = nparts < 65535u ? nparts : 65535u;
    k_part_sums<<<gp, 256, 0, s>>>(per_start, g->rank_l, d_part_l, nparts,
                                   (unsigned long long *)d_totals);
    BFC_HIP(hipGetLastError());
    return BFC_OK;
}

int bfc_autotune_ws_size(const bfc_graph *g, size_t *bytes) {
    if (!g || !bytes) return BFC_E_NULL;
    size_t a = 0, b = 0;
    BFC_TRY(bfc_exact_parts_ws_size(g, &a));
    BFC_TRY(bfc_exact_ws_size(g, BFC_SIDE_AUTO, &b));
    b += 256;
    *bytes = a > b ? a : b;
    return BFC_OK;
}

// Times candidate tunings on this graph (nparts == 0: bfc_exact_tuned with
// the automatic side) or this batch (bfc_exact_parts) and returns the
// fastest.  Three stages: the narrow/wide threshold with the queue chunk,
// the grid shapes for the best of those, then the hash tables of sparse
// starts (off, or at most 16, 64 or 256 wedges per spanned window).  Each candidate runs
// once untimed and three times timed with events on the stream; the minimum
// counts.
int bfc_autotune(const bfc_graph *g, uint32_t nparts, const uint32_t *d_part_l,
                 uint64_t *d_totals, void *d_ws, size_t ws_bytes, hipStream_t s,
                 bfc_tuning *best, float *best_ms) {
    if (!g || !d_ws || !best || !d_totals) return BFC_E_NULL;
    if (nparts && !d_part_l) return BFC_E_NULL;
    size_t need = 0;
    BFC_TRY(bfc_autotune_ws_size(g, &need));
    if (ws_bytes < need) return BFC_E_WS_SMALL;
    hipEvent_t e0, e1;
    BFC_HIP(hipEventCreate(&e0));
    BFC_HIP(hipEventCreate(&e1));
    auto run = [&](const bfc_tuning &t) -> int {
        if (nparts) return bfc_exact_parts(g, nparts, d_part_l, &t, d_totals, d_ws, ws_bytes, s);
        return bfc_exact_tuned(g, BFC_SIDE_AUTO, &t, d_totals, d_ws, ws_bytes, s);
    };
    auto time_one = [&](const bfc_tuning &t, float &ms) -> int {
        BFC_TRY(run(t));
        float bestm = 3.4e38f;
        for (int i = 0; i < 3; i++) {
            BFC_HIP(hipEventRecord(e0, s));
            BFC_TRY(run(t));
            BFC_HIP(hipEventRecord(e1, s));
            BFC_HIP(hipEventSynchronize(e1));
            float x = 0.f;
            BFC_HIP(hipEventElapsedTime(&x, e0, e1));
            if (x < bestm) bestm = x;
        }
        ms = bestm;
        return BFC_OK;
    };
    bfc_tuning cur = {NARROW_MAX, (uint32_t)WCHUNK, 8, 2};
    float cur_ms = 3.4e38f;
    int rc = BFC_OK;
    const uint32_t thresholds[] = {255, 127, 63, 31};
    const uint32_t chunks[] = {1, 4, 16};
    for (uint32_t nm : thresholds)
        for (uint32_t ch : chunks) {
            bfc_tuning t = {nm, ch, 8, 2};
            float ms;
            if ((rc = time_one(t, ms)) != BFC_OK) goto out;
            if (ms < cur_ms) { cur_ms = ms; cur = t; }
        }
    {
        const uint32_t nw[] = {8, 6, 4};
        const uint32_t wg[] = {2, 1};
        const bfc_tuning base = cur;
        for (uint32_t a : nw)
            for (uint32_t b : wg) {
                if (a == base.narrow_waves_per_cu && b == base.wide_groups_per_cu) continue;
                bfc_tuning t = base;
                t.narrow_waves_per_cu = a;
                t.wide_groups_per_cu = b;
                float ms;
                if ((rc = time_one(t, ms)) != BFC_OK) goto out;
                if (ms < cur_ms) { cur_ms = ms; cur = t; }
            }
    }
    {
        // hash tables for sparse starts: off, or up to 16, 32, 64 or 256 wedges per window
        const uint32_t hd[] = {0, 16, 32, 64, 256};
        const bfc_tuning base = cur;
        for (uint32_t d : hd) {
            bfc_tuning t = base;
            if (d == 0) {
                t.hash_small_max = t.hash_mid_max = BFC_HASH_OFF;
            } else {
                t.hash_max_density = d;
            }
            if (d == HASH_DENSITY && base.hash_max_density == 0 && base.hash_small_max == 0)
                continue;                       // the defaults: timed already
            float ms;
            if ((rc = time_one(t, ms)) != BFC_OK) goto out;
            if (ms < cur_ms) { cur_ms = ms; cur = t; }
        }
    }
    *best = cur;
    if (best_ms) *best_ms = cur_ms;
out:
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

// ------------------------------------------------------------------ no-allocation variant
// bfc_exact with its workspace in a static device array: one copy per GPU,
// held until the process ends.  Host code never uses the array's name as an
// address (in host code it is only a stand-in for the symbol); the device
// address of each GPU's copy is looked up once with hipGetSymbolAddress while
// that GPU is current and kept per device.
static __device__ __align__(256) unsigned char scratch[BFC_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
void *scratch_dev[MAX_DEVICES];
}  // namespace

static int scratch_ptr(void **out) {
    int dev = 0;
    BFC_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) return BFC_E_ARG;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_dev[dev]) {
        void *ptr = nullptr;
        BFC_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr || !aligned256(ptr)) return BFC_E_ALIGN;
        scratch_dev[dev] = ptr;
    }
    *out = scratch_dev[dev];
    return BFC_OK;
}

int bfc_exact_noalloc(const bfc_graph *g, int side, uint64_t *d_total, hipStream_t s) {
    if (!g || !d_total) return BFC_E_NULL;
    size_t need = 0;
    BFC_TRY(bfc_exact_ws_size(g, side, &need));
    if (need > (size_t)BFC_NOALLOC_SCRATCH_BYTES) return BFC_E_TOO_LARGE;
    void *ws = nullptr;
    BFC_TRY(scratch_ptr(&ws));
    // every workspace value the count uses is written by this call's plan
    // kernels first (the queue state is cleared by a kernel, not a memset),
    // so what an earlier call left in the array does not matter
    return bfc_exact(g, side, d_total, ws, (size_t)BFC_NOALLOC_SCRATCH_BYTES, s);
}

int bfc_local_ws_size(const bfc_graph *g, size_t *bytes) {
    return bfc::local_ws_size(g, BFC_SIDE_AUTO, bytes, 0);
}

int bfc_local_split_ws_size(const bfc_graph *g, uint64_t split_wedges, size_t *bytes) {
    return bfc::local_ws_size(g, BFC_SIDE_AUTO, bytes, split_wedges);
}

int bfc_local_split(const bfc_graph *g, uint64_t split_wedges, uint64_t *d_cnt_l,
                    uint64_t *d_cnt_r, uint64_t *d_cnt_e, void *d_ws, size_t ws_bytes,
                    hipStream_t s) {
    if (!g || !d_ws || (!d_cnt_l && !d_cnt_r && !d_cnt_e)) return BFC_E_NULL;
    if (((uintptr_t)d_cnt_l & 7) || ((uintptr_t)d_cnt_r & 7) || ((uintptr_t)d_cnt_e & 7))
        return BFC_E_ALIGN;
    unsigned long long *cl = (unsigned long long *)d_cnt_l, *cr = (unsigned long long *)d_cnt_r,
                       *ce = (unsigned long long *)d_cnt_e;
    if (cl) k_zero_u64<<<grid_for(g->n_left), 256, 0, s>>>(cl, g->n_left);
    if (cr) k_zero_u64<<<grid_for(g->n_right), 256, 0, s>>>(cr, g->n_right);
    if (ce) k_zero_u64<<<grid_for(g->n_edges), 256, 0, s>>>(ce, g->n_edges);
    BFC_HIP(hipGetLastError());
    return bfc::local_run(g, BFC_SIDE_AUTO, nullptr, d_cnt_l, d_cnt_r, d_cnt_e, d_ws, ws_bytes, s,
                          split_wedges);
}

int bfc_local(const bfc_graph *g, uint64_t *d_cnt_l, uint64_t *d_cnt_r, uint64_t *d_cnt_e,
              void *d_ws, size_t ws_bytes, hipStream_t s) {
    if (!g || !d_ws || (!d_cnt_l && !d_cnt_r && !d_cnt_e)) return BFC_E_NULL;
    if (((uintptr_t)d_cnt_l & 7) || ((uintptr_t)d_cnt_r & 7) || ((uintptr_t)d_cnt_e & 7))
        return BFC_E_ALIGN;
    unsigned long long *cl = (unsigned long long *)d_cnt_l, *cr = (unsigned long long *)d_cnt_r,
                       *ce = (unsigned long long *)d_cnt_e;
    if (cl) k_zero_u64<<<grid_for(g->n_left), 256, 0, s>>>(cl, g->n_left);
    if (cr) k_zero_u64<<<grid_for(g->n_right), 256, 0, s>>>(cr, g->n_right);
    if (ce) k_zero_u64<<<grid_for(g->n_edges), 256, 0, s>>>(ce, g->n_edges);
    BFC_HIP(hipGetLastError());
    return bfc::local_run(g, BFC_SIDE_AUTO, nullptr, d_cnt_l, d_cnt_r, d_cnt_e, d_ws, ws_bytes, s,
                          0);
}

int bfc_per_vertex(const bfc_graph *g, uint64_t *d_cnt_l, uint64_t *d_cnt_r, void *d_ws,
                   size_t ws_bytes, hipStream_t s) {
    if (!d_cnt_l || !d_cnt_r) return BFC_E_NULL;
    return bfc_local(g, d_cnt_l, d_cnt_r, nullptr, d_ws, ws_bytes, s);
}

int bfc_per_edge(const bfc_graph *g, uint64_t *d_cnt_e, void *d_ws, size_t ws_bytes,
                 hipStream_t s) {
    if (!d_cnt_e) return BFC_E_NULL;
    return bfc_local(g, nullptr, nullptr, d_cnt_e, d_ws, ws_bytes, s);
}

}  // extern "C"
