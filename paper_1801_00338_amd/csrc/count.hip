// Exact butterfly count (ExactBFC, Sec. 4 of the paper) on gfx950.
//
// Work decomposition.  The start side A is chosen by the paper's rule (the
// side whose opposite has the smaller sum of squared degrees is walked as
// midpoints).  For a start u (a rank on side A) every midpoint v in N(u)
// contributes the suffix of adj_B[v] that lies above u; because adjacency
// lists are sorted by rank, that suffix begins right after u's own position
// in adj_B[v] (xpos) and no search is needed.
//
// Counting table.  C_u[w] lives in LDS as a dense window of the rank space:
// with d_u <= 255 every count fits a byte (C_u[w] <= d_u), so a 64 KiB table
// covers 65536 consecutive ranks; wider starts use 32-bit counters over
// 16384 ranks.  Each wedge adds one with a returning LDS atomic, and the old
// value is what the pair {u, w} gains (C(c+1,2) - C(c,2) = c), so the fold
// C(C_u[w], 2) happens as the walk goes.
//
// Windows.  Each adjacency list of B is cut into segments at window
// boundaries (a planning pass).  A start walks its midpoints' suffixes one
// window at a time, in increasing window order, skipping windows no suffix
// touches: per window every midpoint contributes at most one contiguous
// sub-run.  Sub-runs are cut into 16-byte aligned groups of 4 entries, the
// groups of all midpoints are spread over the workgroup's lanes (an LDS
// prefix sum and binary search map a group to its midpoint), and each lane
// does one 16-byte load per group.
//
// Scheduling.  Starts are bucketed by their wedge count (log2) and handed out
// largest first through an atomic queue to a persistent grid.
#include "common.h"

namespace bfc {

constexpr int NT = 256;                 // threads per workgroup
constexpr int TBL_BYTES = 65536;        // LDS counter table
constexpr int G_SHIFT = 16;             // window = 2^16 ranks (byte counters)
constexpr int W32_SHIFT = 14;           // 2^14 ranks with 32-bit counters
constexpr int KEEP = 2;                 // groups per lane kept for the cheap clear
constexpr uint32_t INF = 0xFFFFFFFFu;
constexpr int NBUCKET = 66;

struct Plan {
    int start_r;                        // 0: starts in L, 1: starts in R
    uint32_t nA, nB;
    uint64_t m;
    const uint32_t *offA, *adjA, *xA, *offB, *adjB;
    uint32_t max_deg_A;
    uint64_t wedges;
};

static int make_plan(const bfc_graph *g, int side, Plan *p) {
    if (!g) return BFC_E_NULL;
    int r;
    if (side == BFC_SIDE_AUTO) r = g->sumsq_l < g->sumsq_r;
    else if (side == BFC_SIDE_L) r = 0;
    else if (side == BFC_SIDE_R) r = 1;
    else return BFC_E_ARG;
    p->start_r = r;
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
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < nB; v += gridDim.x * blockDim.x)
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

// Wedges of start u: sum over v in N(u) of the entries of adj_B[v] after u
// (all entries but u itself when `all_ends`, for the local counts).
// Bucket = bit length of that count (0 = nothing to do).
__global__ __launch_bounds__(256) void k_work(const uint32_t *offA, const uint32_t *adjA,
                                              const uint32_t *xA, const uint32_t *offB,
                                              uint32_t nA, int all_ends, uint8_t *bucket,
                                              uint32_t *bcount) {
    __shared__ uint32_t hist[NBUCKET];
    for (int i = threadIdx.x; i < NBUCKET; i += blockDim.x) hist[i] = 0;
    __syncthreads();
    const int lane = threadIdx.x & (WAVE - 1);
    const uint32_t wpb = blockDim.x / WAVE;
    for (uint32_t u = blockIdx.x * wpb + threadIdx.x / WAVE; u < nA; u += gridDim.x * wpb) {
        uint32_t rb = offA[u], re = offA[u + 1];
        unsigned long long t = 0;
        for (uint32_t k = rb + lane; k < re; k += WAVE) {
            uint32_t v = adjA[k];
            t += offB[v + 1] - (all_ends ? offB[v] : xA[k]) - 1;
        }
        t = wave_sum64(t);
        if (lane == 0) {
            uint32_t b = t ? 64 - __clzll(t) : 0;
            bucket[u] = (uint8_t)b;
            if (b) atomicAdd(&hist[b], 1u);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < NBUCKET; i += blockDim.x)
        if (hist[i]) atomicAdd(&bcount[i], hist[i]);
}

// Bucket b's items start after all larger buckets (largest work first).
// Also zeroes the queue head and the output total.
struct QueueState {
    uint32_t bcount[NBUCKET];
    uint32_t cursor[NBUCKET];
    uint32_t n_items;
    uint32_t head;                      // next item to hand out
    uint32_t done;                      // workgroups finished
    uint32_t pad;
    unsigned long long acc;             // running total of the launch
};

// End of a persistent launch: add this workgroup's sum; the last workgroup
// to finish publishes the total and re-arms the queue for the next launch.
__device__ inline void finish_launch(QueueState *q, unsigned long long part,
                                     unsigned long long *total) {
    if (threadIdx.x != 0) return;
    if (part) atomicAdd(&q->acc, part);
    __threadfence();
    uint32_t d = atomicAdd(&q->done, 1u);
    if (d == gridDim.x - 1) {
        __threadfence();
        unsigned long long t = atomicAdd(&q->acc, 0ull);
        if (total) *total = t;
        q->acc = 0;
        q->head = 0;
        q->done = 0;
        __threadfence();
    }
}

__global__ void k_bucket_offsets(QueueState *q, unsigned long long *total) {
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (int b = NBUCKET - 1; b >= 1; b--) {
            q->cursor[b] = run;
            run += q->bcount[b];
        }
        q->n_items = run;
        q->head = 0;
        if (total) *total = 0;
    }
}

__global__ __launch_bounds__(256) void k_scatter_items(const uint8_t *bucket, uint32_t nA,
                                                       QueueState *q, uint32_t *items) {
    __shared__ uint32_t hist[NBUCKET], base[NBUCKET];
    for (int i = threadIdx.x; i < NBUCKET; i += blockDim.x) hist[i] = 0;
    __syncthreads();
    uint32_t u = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t b = 0, local = 0;
    if (u < nA) {
        b = bucket[u];
        if (b) local = atomicAdd(&hist[b], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < NBUCKET; i += blockDim.x)
        if (hist[i]) base[i] = atomicAdd(&q->cursor[i], hist[i]);
    __syncthreads();
    if (b) items[base[b] + local] = u;
}

__global__ void k_zero_u32(uint32_t *p, uint64_t n) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// ------------------------------------------------------------------ the count
struct CountArgs {
    const uint32_t *offA, *adjA, *xA, *offB, *adjB;
    const uint32_t *seg1, *seg_start, *seg_win;
    const uint32_t *items;
    QueueState *q;
    uint32_t nA;
    unsigned long long *total;
};

struct Shared {
    uint32_t tbl[TBL_BYTES / 4];
    uint32_t pre[NT];
    uint32_t lo[NT];
    uint32_t hi[NT];
    uint32_t red[NT / WAVE + 1];
    unsigned long long red64[NT / WAVE];
    uint32_t item;
};

__device__ inline void clear_table(Shared &sh) {
    uint4 z = make_uint4(0, 0, 0, 0);
    for (int i = threadIdx.x; i < TBL_BYTES / 16; i += NT) ((uint4 *)sh.tbl)[i] = z;
}

// Byte counters: add one to counter `off` and return its previous value.
__device__ inline uint32_t bump8(Shared &sh, uint32_t off) {
    uint32_t sh8 = (off & 3u) << 3;
    uint32_t old = atomicAdd(&sh.tbl[off >> 2], 1u << sh8);
    return (old >> sh8) & 0xFFu;
}

__device__ inline void group_bump8(Shared &sh, uint4 q, uint32_t base, uint32_t lo, uint32_t hi,
                                   uint32_t win_base, unsigned long long &sum) {
    uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
    for (int i = 0; i < 4; i++) {
        uint32_t pos = base + i;
        if (pos >= lo && pos < hi) sum += bump8(sh, w[i] - win_base);
    }
}

__device__ inline void group_clear8(Shared &sh, uint4 q, uint32_t base, uint32_t lo, uint32_t hi,
                                    uint32_t win_base) {
    uint32_t w[4] = {q.x, q.y, q.z, q.w};
    uint8_t *t8 = (uint8_t *)sh.tbl;
#pragma unroll
    for (int i = 0; i < 4; i++) {
        uint32_t pos = base + i;
        if (pos >= lo && pos < hi) t8[w[i] - win_base] = 0;
    }
}

// One start with d_u < NT: one midpoint per lane, byte counters, windows of
// 2^16 ranks visited in increasing order, empty windows skipped.
__device__ unsigned long long count_narrow(const CountArgs &a, Shared &sh, uint32_t rb,
                                           uint32_t du) {
    const uint32_t tid = threadIdx.x;
    uint32_t p = 0, ev = 0, cur = 0, win = INF;
    if (tid < du) {
        uint32_t k = rb + tid;
        uint32_t v = a.adjA[k];
        p = a.xA[k] + 1;
        ev = a.offB[v + 1];
        if (p < ev) {
            cur = a.seg1[p] - 1;
            win = a.seg_win[cur];
        }
    }
    unsigned long long sum = 0;
    for (;;) {
        const uint32_t kw = block_min<NT>(win, sh.red);
        if (kw == INF) break;
        uint32_t lo = 0, hi = 0, nch = 0;
        if (win == kw) {
            lo = p;
            uint32_t e = a.seg_start[cur + 1];
            hi = e < ev ? e : ev;
            nch = ((hi + 3) >> 2) - (lo >> 2);
            p = hi;
            if (p < ev) {
                cur++;
                win = a.seg_win[cur];
            } else {
                win = INF;
            }
        }
        uint32_t C;
        uint32_t ex = block_excl_scan<NT>(nch, sh.red, &C);
        sh.pre[tid] = ex;
        sh.lo[tid] = lo;
        sh.hi[tid] = hi;
        __syncthreads();
        const uint32_t wb = kw << G_SHIFT;
        uint4 kq[KEEP];
        uint32_t kb[KEEP], kl[KEEP], kh[KEEP];
#pragma unroll
        for (int r = 0; r < KEEP; r++) {
            uint32_t c = tid + r * NT;
            kl[r] = kh[r] = kb[r] = 0;
            kq[r] = make_uint4(0, 0, 0, 0);
            if (c < C) {
                uint32_t j = upper_bound_lds(sh.pre, du, c) - 1;
                kl[r] = sh.lo[j];
                kh[r] = sh.hi[j];
                kb[r] = ((kl[r] >> 2) + (c - sh.pre[j])) << 2;
                kq[r] = *(const uint4 *)(a.adjB + kb[r]);
            }
        }
#pragma unroll
        for (int r = 0; r < KEEP; r++) group_bump8(sh, kq[r], kb[r], kl[r], kh[r], wb, sum);
        for (uint32_t c = tid + KEEP * NT; c < C; c += NT) {
            uint32_t j = upper_bound_lds(sh.pre, du, c) - 1;
            uint32_t l = sh.lo[j], h = sh.hi[j];
            uint32_t b = ((l >> 2) + (c - sh.pre[j])) << 2;
            uint4 q = *(const uint4 *)(a.adjB + b);
            group_bump8(sh, q, b, l, h, wb, sum);
        }
        __syncthreads();
        if (C <= (uint32_t)(KEEP * NT)) {
#pragma unroll
            for (int r = 0; r < KEEP; r++) group_clear8(sh, kq[r], kb[r], kl[r], kh[r], wb);
        } else {
            clear_table(sh);
        }
        __syncthreads();
    }
    return sum;
}

// One start with d_u >= NT: 32-bit counters over windows of 2^14 ranks,
// midpoints in batches of NT, sub-runs found by binary search.
__device__ unsigned long long count_wide(const CountArgs &a, Shared &sh, uint32_t u, uint32_t rb,
                                         uint32_t du) {
    const uint32_t tid = threadIdx.x;
    unsigned long long sum = 0;
    if (u + 1 >= a.nA) return 0;
    const uint32_t w_first = (u + 1) >> W32_SHIFT, w_last = (a.nA - 1) >> W32_SHIFT;
    for (uint32_t kw = w_first; kw <= w_last; kw++) {
        const uint32_t wb = kw << W32_SHIFT;
        const uint32_t we = wb + (1u << W32_SHIFT);
        for (uint32_t mb = 0; mb < du; mb += NT) {
            uint32_t lo = 0, hi = 0, nch = 0;
            if (mb + tid < du) {
                uint32_t k = rb + mb + tid;
                uint32_t v = a.adjA[k];
                uint32_t p = a.xA[k] + 1, ev = a.offB[v + 1];
                if (p < ev) {
                    lo = lower_bound_glb(a.adjB, p, ev, wb);
                    hi = lower_bound_glb(a.adjB, lo, ev, we);
                    if (hi > lo) nch = ((hi + 3) >> 2) - (lo >> 2);
                }
            }
            uint32_t C;
            uint32_t ex = block_excl_scan<NT>(nch, sh.red, &C);
            sh.pre[tid] = ex;
            sh.lo[tid] = lo;
            sh.hi[tid] = hi;
            __syncthreads();
            for (uint32_t c = tid; c < C; c += NT) {
                uint32_t j = upper_bound_lds(sh.pre, NT, c) - 1;
                uint32_t l = sh.lo[j], h = sh.hi[j];
                uint32_t b = ((l >> 2) + (c - sh.pre[j])) << 2;
                uint4 q = *(const uint4 *)(a.adjB + b);
                uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
                for (int i = 0; i < 4; i++) {
                    uint32_t pos = b + i;
                    if (pos >= l && pos < h) sum += atomicAdd(&sh.tbl[w[i] - wb], 1u);
                }
            }
            __syncthreads();
        }
        clear_table(sh);
        __syncthreads();
    }
    return sum;
}

__global__ __launch_bounds__(NT) void k_exact(CountArgs a) {
    __shared__ Shared sh;
    clear_table(sh);
    __syncthreads();
    unsigned long long acc = 0;
    const uint32_t n_items = a.q->n_items;
    for (;;) {
        if (threadIdx.x == 0) sh.item = atomicAdd(&a.q->head, 1u);
        __syncthreads();
        const uint32_t it = sh.item;
        __syncthreads();
        if (it >= n_items) break;
        const uint32_t u = a.items[it];
        const uint32_t rb = a.offA[u], du = a.offA[u + 1] - rb;
        if (du < (uint32_t)NT) acc += count_narrow(a, sh, rb, du);
        else acc += count_wide(a, sh, u, rb, du);
    }
    acc = block_sum64<NT>(acc, sh.red64);
    finish_launch(a.q, acc, a.total);
}

// ------------------------------------------------------------------ local counts
// For a start u the walk takes every endpoint w != u (no order), so C_u[w] =
// |N(u) & N(w)| for all same-side w and
//   B_u       = sum_w C(C_u[w], 2)                       (Eq. (2))
//   B_(u,v)   = sum_{w in N(v), w != u} (C_u[w] - 1)       (edge definition)
//   B_v (mid) = 1/2 sum_{u in N(v)} B_(u,v)               (two edges of v per butterfly)
// The first sum runs during the increments; after a window's increments the
// same entries are read again and summed per midpoint.
struct LocalArgs {
    CountArgs c;
    const uint32_t *eidA, *idA;
    unsigned long long *cntA;     // per start-side vertex (caller ids), or null
    unsigned long long *cntE;     // per edge (caller order), or null
    unsigned long long *twiceB;   // 2 B_v per midpoint rank (workspace)
    unsigned long long *esum;     // per A-side CSR position (workspace, wide starts)
};

struct LocalShared {
    Shared s;
    uint32_t x[NT];
    unsigned long long esum[NT];
};

__device__ inline void group_read8(const Shared &sh, uint4 q, uint32_t base, uint32_t lo,
                                   uint32_t hi, uint32_t skip, uint32_t win_base,
                                   unsigned long long &acc) {
    uint32_t w[4] = {q.x, q.y, q.z, q.w};
    const uint8_t *t8 = (const uint8_t *)sh.tbl;
#pragma unroll
    for (int i = 0; i < 4; i++) {
        uint32_t pos = base + i;
        if (pos >= lo && pos < hi && pos != skip) acc += t8[w[i] - win_base];
    }
}

__device__ inline void group_bump8_skip(Shared &sh, uint4 q, uint32_t base, uint32_t lo,
                                        uint32_t hi, uint32_t skip, uint32_t win_base,
                                        unsigned long long &sum) {
    uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
    for (int i = 0; i < 4; i++) {
        uint32_t pos = base + i;
        if (pos >= lo && pos < hi && pos != skip) sum += bump8(sh, w[i] - win_base);
    }
}

__device__ inline void group_clear8_skip(Shared &sh, uint4 q, uint32_t base, uint32_t lo,
                                         uint32_t hi, uint32_t skip, uint32_t win_base) {
    uint32_t w[4] = {q.x, q.y, q.z, q.w};
    uint8_t *t8 = (uint8_t *)sh.tbl;
#pragma unroll
    for (int i = 0; i < 4; i++) {
        uint32_t pos = base + i;
        if (pos >= lo && pos < hi && pos != skip) t8[w[i] - win_base] = 0;
    }
}

__device__ void local_narrow(const LocalArgs &a, LocalShared &ls, uint32_t u, uint32_t rb,
                             uint32_t du) {
    Shared &sh = ls.s;
    const CountArgs &c = a.c;
    const uint32_t tid = threadIdx.x;
    uint32_t p = 0, ev = 0, cur = 0, win = INF, v = 0, x = 0;
    if (tid < du) {
        uint32_t k = rb + tid;
        v = c.adjA[k];
        x = c.xA[k];
        p = c.offB[v];
        ev = c.offB[v + 1];
        if (ev - p > 1) {                 // some endpoint other than u
            cur = c.seg1[p] - 1;
            win = c.seg_win[cur];
        }
        ls.x[tid] = x;
    }
    ls.esum[tid] = 0;
    unsigned long long sum = 0;
    for (;;) {
        const uint32_t kw = block_min<NT>(win, sh.red);
        if (kw == INF) break;
        uint32_t lo = 0, hi = 0, nch = 0;
        if (win == kw) {
            lo = p;
            uint32_t e = c.seg_start[cur + 1];
            hi = e < ev ? e : ev;
            nch = ((hi + 3) >> 2) - (lo >> 2);
            p = hi;
            if (p < ev) {
                cur++;
                win = c.seg_win[cur];
            } else {
                win = INF;
            }
        }
        uint32_t C;
        uint32_t ex = block_excl_scan<NT>(nch, sh.red, &C);
        sh.pre[tid] = ex;
        sh.lo[tid] = lo;
        sh.hi[tid] = hi;
        __syncthreads();
        const uint32_t wb = kw << G_SHIFT;
        uint4 kq[KEEP];
        uint32_t kb[KEEP], kj[KEEP];
        bool kv[KEEP];
#pragma unroll
        for (int r = 0; r < KEEP; r++) {
            uint32_t cc = tid + r * NT;
            kv[r] = cc < C;
            kb[r] = kj[r] = 0;
            kq[r] = make_uint4(0, 0, 0, 0);
            if (kv[r]) {
                uint32_t j = upper_bound_lds(sh.pre, du, cc) - 1;
                kj[r] = j;
                kb[r] = ((sh.lo[j] >> 2) + (cc - sh.pre[j])) << 2;
                kq[r] = *(const uint4 *)(c.adjB + kb[r]);
            }
        }
#pragma unroll
        for (int r = 0; r < KEEP; r++)
            if (kv[r]) {
                uint32_t j = kj[r];
                group_bump8_skip(sh, kq[r], kb[r], sh.lo[j], sh.hi[j], ls.x[j], wb, sum);
            }
        for (uint32_t cc = tid + KEEP * NT; cc < C; cc += NT) {
            uint32_t j = upper_bound_lds(sh.pre, du, cc) - 1;
            uint32_t b = ((sh.lo[j] >> 2) + (cc - sh.pre[j])) << 2;
            uint4 q = *(const uint4 *)(c.adjB + b);
            group_bump8_skip(sh, q, b, sh.lo[j], sh.hi[j], ls.x[j], wb, sum);
        }
        __syncthreads();
        // second look: final counts of this window, summed per midpoint
#pragma unroll
        for (int r = 0; r < KEEP; r++)
            if (kv[r]) {
                uint32_t j = kj[r];
                unsigned long long acc = 0;
                group_read8(sh, kq[r], kb[r], sh.lo[j], sh.hi[j], ls.x[j], wb, acc);
                if (acc) atomicAdd(&ls.esum[j], acc);
            }
        for (uint32_t cc = tid + KEEP * NT; cc < C; cc += NT) {
            uint32_t j = upper_bound_lds(sh.pre, du, cc) - 1;
            uint32_t b = ((sh.lo[j] >> 2) + (cc - sh.pre[j])) << 2;
            uint4 q = *(const uint4 *)(c.adjB + b);
            unsigned long long acc = 0;
            group_read8(sh, q, b, sh.lo[j], sh.hi[j], ls.x[j], wb, acc);
            if (acc) atomicAdd(&ls.esum[j], acc);
        }
        __syncthreads();
        if (C <= (uint32_t)(KEEP * NT)) {
#pragma unroll
            for (int r = 0; r < KEEP; r++)
                if (kv[r]) {
                    uint32_t j = kj[r];
                    group_clear8_skip(sh, kq[r], kb[r], sh.lo[j], sh.hi[j], ls.x[j], wb);
                }
        } else {
            clear_table(sh);
        }
        __syncthreads();
    }
    if (tid < du) {
        unsigned long long e = ls.esum[tid] - (unsigned long long)(ev - c.offB[v] - 1);
        if (a.cntE) a.cntE[a.eidA[rb + tid]] = e;
        if (e) atomicAdd(&a.twiceB[v], e);
    }
    sum = block_sum64<NT>(sum, sh.red64);
    if (tid == 0 && a.cntA) a.cntA[a.idA[u]] = sum;
}

__device__ void local_wide(const LocalArgs &a, LocalShared &ls, uint32_t u, uint32_t rb,
                           uint32_t du) {
    Shared &sh = ls.s;
    const CountArgs &c = a.c;
    const uint32_t tid = threadIdx.x;
    unsigned long long sum = 0;
    for (uint32_t mb = tid; mb < du; mb += NT) a.esum[rb + mb] = 0;
    const uint32_t w_last = (c.nA - 1) >> W32_SHIFT;
    for (uint32_t kw = 0; kw <= w_last; kw++) {
        const uint32_t wb = kw << W32_SHIFT;
        const uint32_t we = wb + (1u << W32_SHIFT);
        for (int pass = 0; pass < 2; pass++) {
            for (uint32_t mb = 0; mb < du; mb += NT) {
                uint32_t lo = 0, hi = 0, nch = 0, x = 0;
                if (mb + tid < du) {
                    uint32_t k = rb + mb + tid;
                    uint32_t v = c.adjA[k];
                    uint32_t pb = c.offB[v], ev = c.offB[v + 1];
                    x = c.xA[k];
                    lo = lower_bound_glb(c.adjB, pb, ev, wb);
                    hi = lower_bound_glb(c.adjB, lo, ev, we);
                    if (hi > lo) nch = ((hi + 3) >> 2) - (lo >> 2);
                }
                uint32_t C;
                uint32_t ex = block_excl_scan<NT>(nch, sh.red, &C);
                sh.pre[tid] = ex;
                sh.lo[tid] = lo;
                sh.hi[tid] = hi;
                ls.x[tid] = x;
                ls.esum[tid] = 0;
                __syncthreads();
                uint32_t nm = du - mb < (uint32_t)NT ? du - mb : (uint32_t)NT;
                for (uint32_t cc = tid; cc < C; cc += NT) {
                    uint32_t j = upper_bound_lds(sh.pre, nm, cc) - 1;
                    uint32_t l = sh.lo[j], h = sh.hi[j], sk = ls.x[j];
                    uint32_t b = ((l >> 2) + (cc - sh.pre[j])) << 2;
                    uint4 q = *(const uint4 *)(c.adjB + b);
                    uint32_t w[4] = {q.x, q.y, q.z, q.w};
                    unsigned long long acc = 0;
#pragma unroll
                    for (int i = 0; i < 4; i++) {
                        uint32_t pos = b + i;
                        if (pos >= l && pos < h && pos != sk) {
                            if (pass == 0) sum += atomicAdd(&sh.tbl[w[i] - wb], 1u);
                            else acc += sh.tbl[w[i] - wb];
                        }
                    }
                    if (pass == 1 && acc) atomicAdd(&ls.esum[j], acc);
                }
                __syncthreads();
                if (pass == 1 && mb + tid < du) a.esum[rb + mb + tid] += ls.esum[tid];
                __syncthreads();
            }
        }
        clear_table(sh);
        __syncthreads();
    }
    for (uint32_t j = tid; j < du; j += NT) {
        uint32_t k = rb + j;
        uint32_t v = c.adjA[k];
        unsigned long long e = a.esum[k] - (unsigned long long)(c.offB[v + 1] - c.offB[v] - 1);
        if (a.cntE) a.cntE[a.eidA[k]] = e;
        if (e) atomicAdd(&a.twiceB[v], e);
    }
    sum = block_sum64<NT>(sum, sh.red64);
    if (tid == 0 && a.cntA) a.cntA[a.idA[u]] = sum;
}

__global__ __launch_bounds__(NT) void k_local(LocalArgs a) {
    __shared__ LocalShared ls;
    clear_table(ls.s);
    __syncthreads();
    const uint32_t n_items = a.c.q->n_items;
    for (;;) {
        if (threadIdx.x == 0) ls.s.item = atomicAdd(&a.c.q->head, 1u);
        __syncthreads();
        const uint32_t it = ls.s.item;
        __syncthreads();
        if (it >= n_items) break;
        const uint32_t u = a.c.items[it];
        const uint32_t rb = a.c.offA[u], du = a.c.offA[u + 1] - rb;
        if (du < (uint32_t)NT) local_narrow(a, ls, u, rb, du);
        else local_wide(a, ls, u, rb, du);
    }
    finish_launch(a.c.q, 0, nullptr);
}

// B_v of the midpoint side from the edge sums; outputs in caller ids.
__global__ void k_local_finish(const unsigned long long *twiceB, const uint32_t *idB, uint32_t nB,
                               unsigned long long *cntB) {
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < nB; v += gridDim.x * blockDim.x)
        cntB[idB[v]] = twiceB[v] >> 1;
}

__global__ void k_zero_u64(unsigned long long *p, uint64_t n) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// ------------------------------------------------------------------ host side
struct ExactWs {
    uint32_t *seg1, *seg_start, *seg_win, *scan_tmp, *items;
    uint8_t *bucket;
    QueueState *q;
};

static ExactWs carve_exact(Carver &c, const Plan &p) {
    ExactWs w;
    w.seg1 = c.take<uint32_t>(pad64(p.m));
    w.seg_start = c.take<uint32_t>(pad64(p.m + 1));
    w.seg_win = c.take<uint32_t>(pad64(p.m));
    w.scan_tmp = c.take<uint32_t>(scan_tmp_elems(p.m));
    w.items = c.take<uint32_t>(pad64(p.nA));
    w.bucket = c.take<uint8_t>(pad64(p.nA));
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
static bool overflow_risk(const Plan &p) {
    if (p.max_deg_A < 2) return false;
    unsigned __int128 b = (unsigned __int128)p.wedges * (p.max_deg_A - 1) / 2;
    return b >> 64;
}

// Segments, per-start work buckets and the work queue for one plan.
static int prepare(const Plan &p, ExactWs &w, unsigned long long *d_total, int all_ends,
                   hipStream_t s) {
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(256), 0, s, (uint32_t *)w.q,
                       (uint64_t)(sizeof(QueueState) / 4));
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
        k_work<<<g, 256, 0, s>>>(p.offA, p.adjA, p.xA, p.offB, p.nA, all_ends, w.bucket,
                                 w.q->bcount);
        BFC_HIP(hipGetLastError());
    }
    k_bucket_offsets<<<1, 64, 0, s>>>(w.q, d_total);
    if (p.nA) k_scatter_items<<<grid_for(p.nA), 256, 0, s>>>(w.bucket, p.nA, w.q, w.items);
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

static int exact_setup(const bfc_graph *g, int side, void *d_ws, size_t ws_bytes, Plan &p,
                       ExactWs &w) {
    if (!d_ws) return BFC_E_NULL;
    BFC_TRY(make_plan(g, side, &p));
    if (!aligned256(d_ws)) return BFC_E_ALIGN;
    if (overflow_risk(p)) return BFC_E_OVERFLOW_RISK;
    Carver c(d_ws, ws_bytes);
    w = carve_exact(c, p);
    if (!c.fits()) return BFC_E_WS_SMALL;
    return BFC_OK;
}

int bfc_exact_plan(const bfc_graph *g, int side, void *d_ws, size_t ws_bytes, hipStream_t s) {
    Plan p;
    ExactWs w;
    BFC_TRY(exact_setup(g, side, d_ws, ws_bytes, p, w));
    return prepare(p, w, nullptr, 0, s);
}

int bfc_exact_count(const bfc_graph *g, int side, uint64_t *d_total, void *d_ws,
                    size_t ws_bytes, hipStream_t s) {
    if (!d_total) return BFC_E_NULL;
    if ((uintptr_t)d_total & 7) return BFC_E_ALIGN;
    Plan p;
    ExactWs w;
    BFC_TRY(exact_setup(g, side, d_ws, ws_bytes, p, w));
    unsigned long long *tot = (unsigned long long *)d_total;
    if (p.nA == 0 || p.m == 0) {
        k_zero_u64<<<1, 64, 0, s>>>(tot, 1);
        BFC_HIP(hipGetLastError());
        return BFC_OK;
    }
    CountArgs a;
    a.offA = p.offA; a.adjA = p.adjA; a.xA = p.xA; a.offB = p.offB; a.adjB = p.adjB;
    a.seg1 = w.seg1; a.seg_start = w.seg_start; a.seg_win = w.seg_win;
    a.items = w.items; a.q = w.q; a.nA = p.nA; a.total = tot;
    int dev = 0;
    BFC_HIP(hipGetDevice(&dev));
    unsigned grid = (unsigned)device_cu_count(dev) * 2;
    k_exact<<<grid, NT, 0, s>>>(a);
    BFC_HIP(hipGetLastError());
    return BFC_OK;
}

int bfc_exact(const bfc_graph *g, int side, uint64_t *d_total, void *d_ws, size_t ws_bytes,
              hipStream_t s) {
    if (!d_total) return BFC_E_NULL;
    BFC_TRY(bfc_exact_plan(g, side, d_ws, ws_bytes, s));
    return bfc_exact_count(g, side, d_total, d_ws, ws_bytes, s);
}

}  // extern "C"

namespace bfc {

struct LocalWs {
    ExactWs e;
    unsigned long long *twiceB, *esum;
};

static LocalWs carve_local(Carver &c, const Plan &p) {
    LocalWs w;
    w.e = carve_exact(c, p);
    w.twiceB = c.take<unsigned long long>(pad64(p.nB));
    w.esum = c.take<unsigned long long>(pad64(p.m));
    return w;
}

}  // namespace bfc

extern "C" {

int bfc_local_ws_size(const bfc_graph *g, size_t *bytes) {
    if (!bytes) return BFC_E_NULL;
    Plan p;
    BFC_TRY(make_plan(g, BFC_SIDE_AUTO, &p));
    Carver c(nullptr, 0);
    carve_local(c, p);
    *bytes = c.used;
    return BFC_OK;
}

int bfc_local(const bfc_graph *g, uint64_t *d_cnt_l, uint64_t *d_cnt_r, uint64_t *d_cnt_e,
              void *d_ws, size_t ws_bytes, hipStream_t s) {
    if (!d_ws || (!d_cnt_l && !d_cnt_r && !d_cnt_e)) return BFC_E_NULL;
    Plan p;
    BFC_TRY(make_plan(g, BFC_SIDE_AUTO, &p));
    if (!aligned256(d_ws) || ((uintptr_t)d_cnt_l & 7) || ((uintptr_t)d_cnt_r & 7) ||
        ((uintptr_t)d_cnt_e & 7))
        return BFC_E_ALIGN;
    {
        Plan q = p;
        q.wedges = 2 * p.wedges;
        if (p.wedges >> 63 || overflow_risk(q)) return BFC_E_OVERFLOW_RISK;
    }
    Carver c(d_ws, ws_bytes);
    LocalWs w = carve_local(c, p);
    if (!c.fits()) return BFC_E_WS_SMALL;
    unsigned long long *cl = (unsigned long long *)d_cnt_l, *cr = (unsigned long long *)d_cnt_r,
                       *ce = (unsigned long long *)d_cnt_e;
    if (cl) k_zero_u64<<<grid_for(g->n_left), 256, 0, s>>>(cl, g->n_left);
    if (cr) k_zero_u64<<<grid_for(g->n_right), 256, 0, s>>>(cr, g->n_right);
    if (ce) k_zero_u64<<<grid_for(p.m), 256, 0, s>>>(ce, p.m);
    k_zero_u64<<<grid_for(p.nB), 256, 0, s>>>(w.twiceB, p.nB);
    BFC_HIP(hipGetLastError());
    BFC_TRY(prepare(p, w.e, nullptr, 1, s));
    if (p.nA == 0 || p.m == 0) return BFC_OK;
    LocalArgs a;
    a.c.offA = p.offA; a.c.adjA = p.adjA; a.c.xA = p.xA; a.c.offB = p.offB; a.c.adjB = p.adjB;
    a.c.seg1 = w.e.seg1; a.c.seg_start = w.e.seg_start; a.c.seg_win = w.e.seg_win;
    a.c.items = w.e.items; a.c.q = w.e.q; a.c.nA = p.nA; a.c.total = nullptr;
    a.eidA = p.start_r ? g->eid_r : g->eid_l;
    a.idA = p.start_r ? g->id_r : g->id_l;
    a.cntA = p.start_r ? cr : cl;
    a.cntE = ce;
    a.twiceB = w.twiceB;
    a.esum = w.esum;
    int dev = 0;
    BFC_HIP(hipGetDevice(&dev));
    unsigned grid = (unsigned)device_cu_count(dev) * 2;
    k_local<<<grid, NT, 0, s>>>(a);
    unsigned long long *cntB = p.start_r ? cl : cr;
    if (cntB)
        k_local_finish<<<grid_for(p.nB), 256, 0, s>>>(w.twiceB, p.start_r ? g->id_l : g->id_r,
                                                       p.nB, cntB);
    BFC_HIP(hipGetLastError());
    return BFC_OK;
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
