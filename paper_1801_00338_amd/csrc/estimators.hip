// Estimators built on the exact and local counts (Sec. 5 and 6 of the paper):
// edge sparsification (ESpar), colourful sparsification (ClrSpar), vertex
// sampling (VSamp), edge sampling (ESamp, also with Fast-eBFC) and wedge
// sampling (WSamp).
//
// Random decisions come from Philox-4x32-10 (Salmon, Moraes, Dror, Shaw,
// SC'11) keyed by the 64-bit seed (key = seed low word, seed high word); each
// decision has a fixed counter, so results do not depend on thread order:
//   ESpar keep of edge (l, r):   counter (l, r, 'ESPR', 0), x = out0 | out1 << 32,
//                                kept iff x < floor(p * 2^64)  (p = 1 keeps all)
//   ClrSpar colour of vertex v of side s (0 = L, 1 = R):
//                                counter (v, s, 'CLRS', attempt), x = out0,
//                                rejected while x >= 2^32 - 2^32 mod N, colour x mod N
//   draw i of VSamp / ESamp:     counter (i lo, i hi, 'VDRW' / 'EDRW', attempt),
//                                x = out0 | out1 << 32, rejected while
//                                x >= 2^64 - 2^64 mod n, value x mod n
//   trial j of Fast-eBFC draw i: counter (i, j, 'FEBC', attempt), x1 = out0 | out1 << 32,
//                                x2 = out2 | out3 << 32, both rejected as above
//                                (bounds d_x and d_a), neighbour picks x1 mod d_x
//                                and x2 mod d_a in ascending rank order
//   draw i of WSamp:             counter (i lo, i hi, 'WDRW', attempt), a wedge
//                                number below W, rejected as above
// Weighted draws quantise probabilities to integer weights
// q_j = prob_j > 0 ? max(1, floor(prob_j / max(prob) * (2^32 - 1))) : 0 and
// pick the first j whose inclusive prefix sum of q exceeds a uniform draw
// below the total Q.
#include "common.h"

#include <vector>

namespace bfc {

constexpr uint32_t TAG_ESPAR = 0x45535052u;
constexpr uint32_t TAG_COLOR = 0x434C5253u;
constexpr uint32_t TAG_VDRAW = 0x56445257u;
constexpr uint32_t TAG_EDRAW = 0x45445257u;
constexpr uint32_t TAG_FAST = 0x46454243u;
constexpr uint32_t TAG_WDRAW = 0x57445257u;
constexpr uint32_t COMBINE_BLOCK = 1024;   // draws summed left to right per block

// ------------------------------------------------------------------ Philox
__device__ inline void philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint64_t seed,
                              uint32_t out[4]) {
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
#pragma unroll
    for (int r = 0; r < 10; r++) {
        const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
        const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

// Uniform value below n (n >= 1) by rejection.
__device__ inline uint64_t draw_below(uint64_t seed, uint32_t a, uint32_t b, uint32_t tag,
                                      uint64_t n) {
    const uint64_t rem = (0 - n) % n;         // 2^64 mod n
    uint32_t o[4];
    for (uint32_t attempt = 0;; attempt++) {
        philox(a, b, tag, attempt, seed, o);
        const uint64_t x = (uint64_t)o[0] | ((uint64_t)o[1] << 32);
        if (rem == 0 || x < 0 - rem) return x % n;
    }
}

__device__ inline uint32_t colour_of(uint64_t seed, uint32_t side, uint32_t v, uint32_t N) {
    const uint64_t lim = (0x100000000ull / N) * N;
    uint32_t o[4];
    for (uint32_t attempt = 0;; attempt++) {
        philox(v, side, TAG_COLOR, attempt, seed, o);
        if ((uint64_t)o[0] < lim) return o[0] % N;
    }
}

// ------------------------------------------------------------------ sparsifier kernels
// A sparsifier keeps a subset of the edges, and its estimate is the exact
// count of the kept graph.  The kept graph is built without sorting:
// filtering a CSR row keeps its order, and the ranks restricted to the
// vertices that keep an edge are still a strict total order (any such order
// counts every same-side pair once), so the kept graph's CSRs are
// compactions of the graph's own, each kept vertex renumbered to the number
// of kept vertices ranked below it.

// One replica's keep rule: ESpar by a Philox threshold on the edge's ids,
// ClrSpar by equal colours of its ends.
struct KeepRule {
    int kind;                   // 0 = ESpar, 1 = ClrSpar
    int keep_all;               // p = 1 or N = 1
    uint64_t seed, thresh;      // ESpar: keep iff x < thresh
    const uint32_t *col_l, *col_r;  // ClrSpar colours by rank
};

// One side of the graph as the kept-graph builder reads it.
struct SideView {
    const uint32_t *off, *adj, *xpos;   // rows by rank, neighbour ranks, cross positions
    const uint32_t *id, *id_o;          // ids of this side's and the other side's ranks
    uint32_t n;
    int is_r;                           // rows are R vertices (the rule takes (l, r))
};

// Keep decision of the edge between this side's rank u and the other
// side's rank w.
__device__ inline uint32_t keep_edge(const KeepRule &k, const SideView &v, uint32_t u,
                                     uint32_t w) {
    if (k.keep_all) return 1u;
    if (k.kind == 0) {
        const uint32_t a = v.id[u], b = v.id_o[w];
        uint32_t o[4];
        philox(v.is_r ? b : a, v.is_r ? a : b, TAG_ESPAR, 0, k.seed, o);
        const uint64_t x = (uint64_t)o[0] | ((uint64_t)o[1] << 32);
        return x < k.thresh;
    }
    return v.is_r ? k.col_r[u] == k.col_l[w] : k.col_l[u] == k.col_r[w];
}

// Row of every CSR position of one side (one wave per row; once per call).
__global__ __launch_bounds__(256) void k_row_of(const uint32_t *off, uint32_t n, uint32_t *row) {
    const uint32_t lane = threadIdx.x & (WAVE - 1), wpb = blockDim.x / WAVE;
    for (uint32_t u = blockIdx.x * wpb + threadIdx.x / WAVE; u < n; u += gridDim.x * wpb)
        for (uint32_t p = off[u] + lane; p < off[u + 1]; p += WAVE) row[p] = u;
}

// Keep flag of every CSR position of one side, one thread per position.
__global__ __launch_bounds__(256) void k_keep_flags(SideView v, KeepRule k, const uint32_t *row,
                                                    uint64_t m, uint32_t *flag) {
    for (uint64_t p = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; p < m;
         p += (uint64_t)gridDim.x * blockDim.x)
        flag[p] = keep_edge(k, v, row[p], v.adj[p]);
}

// Kept entries of row u, from the inclusive scan of the keep flags.
__device__ inline uint32_t kept_in_row(const uint32_t *off, const uint32_t *scan, uint32_t u) {
    const uint32_t rb = off[u], re = off[u + 1];
    return (re ? scan[re - 1] : 0u) - (rb ? scan[rb - 1] : 0u);
}

// mark[u] = 1 when row u keeps an edge.
__global__ void k_kept_marks(const uint32_t *off, uint32_t n, const uint32_t *scan,
                             uint32_t *mark) {
    for (uint64_t u = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; u < n;
         u += (uint64_t)gridDim.x * blockDim.x)
        mark[u] = kept_in_row(off, scan, (uint32_t)u) != 0u;
}

// out[0] += rows that keep an edge, out[1] += sum of squared kept degrees.
__global__ __launch_bounds__(256) void k_kept_stats(const uint32_t *off, uint32_t n,
                                                    const uint32_t *scan,
                                                    unsigned long long *out) {
    __shared__ unsigned long long red[256 / WAVE];
    unsigned long long c = 0, q = 0;
    for (uint64_t u = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; u < n;
         u += (uint64_t)gridDim.x * blockDim.x) {
        const unsigned long long d = kept_in_row(off, scan, (uint32_t)u);
        c += d != 0;
        q += d * d;
    }
    c = block_sum64<256>(c, red);
    q = block_sum64<256>(q, red);
    if (threadIdx.x == 0) {
        if (c) atomicAdd(&out[0], c);
        if (q) atomicAdd(&out[1], q);
    }
}

// One side's kept rows written into a CSR (one part of a union, or the whole
// kept graph): the row of new rank r at out_off[vbase + r], its entries at
// ebase + their kept index, each the neighbour's new rank plus vbase_o and,
// when out_xpos is given, the position of the same edge in the other side's
// output.  Nothing is written once *bad is set (a part whose sizes differ
// from those its buffers were sized for).  Offsets one thread per row,
// entries one thread per position.
struct EmitArgs {
    const uint32_t *off, *adj, *xpos;   // source side
    const uint32_t *scan, *scan_o;      // keep-flag scans: this side's order, the other side's
    const uint32_t *vscan, *vscan_o;    // kept-vertex mark scans: this side, the other side
    uint32_t n;
    uint64_t ebase;
    uint32_t vbase, vbase_o;
    uint32_t *out_off, *out_adj, *out_xpos;
    const uint32_t *bad;
};

__global__ __launch_bounds__(256) void k_emit_offsets(EmitArgs a) {
    if (a.bad && *a.bad) return;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < a.n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t u = (uint32_t)i;
        const uint32_t rb = a.off[u], re = a.off[u + 1];
        const uint32_t s0 = rb ? a.scan[rb - 1] : 0u;
        const uint32_t s1 = re ? a.scan[re - 1] : 0u;
        if (s1 != s0) a.out_off[a.vbase + a.vscan[u] - 1] = (uint32_t)(a.ebase + s0);
    }
}

__global__ __launch_bounds__(256) void k_emit_entries(EmitArgs a, uint64_t m) {
    if (a.bad && *a.bad) return;
    for (uint64_t p = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; p < m;
         p += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t inc = a.scan[p], prev = p ? a.scan[p - 1] : 0u;
        if (inc != prev) {
            const uint64_t q = a.ebase + prev;
            a.out_adj[q] = a.vbase_o + a.vscan_o[a.adj[p]] - 1u;
            if (a.out_xpos) a.out_xpos[q] = (uint32_t)(a.ebase + a.scan_o[a.xpos[p]] - 1u);
        }
    }
}

// Tail of a kept graph laid out on the graph's own sizes (the single
// sparsifier calls, whose kept sizes stay on the device): rows from the kept
// vertex count to n end at the kept edge count, and adjacency positions from
// the kept edge count to m hold a rank no vertex has, so the count's
// planning starts a segment there.
__global__ void k_kept_tail(uint32_t *off, uint32_t n, const uint32_t *vscan,
                            const uint32_t *escan, uint64_t m, uint32_t *adj) {
    const uint32_t nk = n ? vscan[n - 1] : 0u;
    const uint32_t mk = m ? escan[m - 1] : 0u;
    const uint64_t lim = (uint64_t)n + 1 > m ? (uint64_t)n + 1 : m;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < lim;
         i += (uint64_t)gridDim.x * blockDim.x) {
        if (i <= n && i >= nk) off[i] = mk;
        if (i < m && i >= mk) adj[i] = 0xFFFFFFFFu;
    }
}

__global__ void k_kept_total(const uint32_t *escan, uint64_t m, unsigned long long *out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *out = m ? escan[m - 1] : 0u;
}

// ClrSpar colours of one side by rank (the colour is drawn for the id).
__global__ void k_colours(uint32_t n, uint32_t side, uint32_t N, uint64_t seed,
                          const uint32_t *id, uint32_t *col) {
    for (uint64_t r = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; r < n;
         r += (uint64_t)gridDim.x * blockDim.x)
        col[r] = colour_of(seed, side, id[r], N);
}

__global__ void k_est_scale(const unsigned long long *beta, double scale_div, double scale_mul,
                            double *est) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double b = (double)*beta;
        *est = scale_div != 0.0 ? b / scale_div : b * scale_mul;
    }
}

// ------------------------------------------------------------------ sampler kernels
struct ProbFlags {
    unsigned long long max_bits;   // bit pattern of the largest probability (all >= 0)
    uint32_t bad;                  // some probability is negative, NaN or infinite
    uint32_t overflow;             // the uniform combine's sum overflowed
};

__global__ void k_prob_scan(const double *probs, uint64_t n, ProbFlags *f) {
    unsigned long long mx = 0;
    uint32_t bad = 0;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const double p = probs[i];
        if (!(p >= 0.0) || isinf(p)) bad = 1;
        else if (p > 0.0) mx = max(mx, (unsigned long long)__double_as_longlong(p));
    }
    if (bad) atomicOr(&f->bad, 1u);
    if (mx) atomicMax(&f->max_bits, mx);
}

// Probabilities that fail the check (negative, NaN, infinite, all zero) are
// replaced by equal weights, so the draws that follow stay well defined; the
// estimate is then NaN (probs_ok below).
__device__ inline bool probs_ok(const ProbFlags *f) { return !f->bad && f->max_bits != 0; }

// Integer weights into w and pre (pre is then scanned in place).
__global__ void k_quantise(const double *probs, uint64_t n, const ProbFlags *f,
                           unsigned long long *w, unsigned long long *pre) {
    const bool ok = probs_ok(f);
    const double mx = __longlong_as_double((long long)f->max_bits);
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const double p = probs[i];
        unsigned long long q = ok ? 0 : 1;
        if (ok && p > 0.0) {
            const double s = floor(p / mx * 4294967295.0);
            const uint32_t v = (uint32_t)s;
            q = v < 1 ? 1 : v;
        }
        w[i] = q;
        pre[i] = q;
    }
}

__global__ void k_zero_flags(ProbFlags *f) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        f->max_bits = 0;
        f->bad = 0;
        f->overflow = 0;
    }
}

__device__ inline double nan64() { return __longlong_as_double(0x7FF8000000000000ll); }

// Inclusive prefix sum of uint64 (same reduce-then-scan as the uint32 scan).
constexpr int S64_NT = 256, S64_PER = 8, S64_TILE = S64_NT * S64_PER;

__global__ __launch_bounds__(S64_NT) void k_s64_tile(const unsigned long long *in, uint64_t n,
                                                     unsigned long long *sums) {
    __shared__ unsigned long long red[S64_NT / WAVE];
    const uint64_t base = (uint64_t)blockIdx.x * S64_TILE;
    unsigned long long s = 0;
    for (int i = 0; i < S64_PER; i++) {
        const uint64_t idx = base + (uint64_t)i * S64_NT + threadIdx.x;
        if (idx < n) s += in[idx];
    }
    s = block_sum64<S64_NT>(s, red);
    if (threadIdx.x == 0) sums[blockIdx.x] = s;
}

__global__ void k_s64_sums(unsigned long long *sums, uint32_t nt) {
    if (threadIdx.x == 0) {
        unsigned long long run = 0;
        for (uint32_t i = 0; i < nt; i++) {
            const unsigned long long v = sums[i];
            sums[i] = run;
            run += v;
        }
    }
}

__global__ __launch_bounds__(S64_NT) void k_s64_apply(unsigned long long *io, uint64_t n,
                                                      const unsigned long long *offs) {
    __shared__ unsigned long long wsum[S64_NT / WAVE];
    const uint64_t base = (uint64_t)blockIdx.x * S64_TILE + (uint64_t)threadIdx.x * S64_PER;
    unsigned long long v[S64_PER], s = 0;
#pragma unroll
    for (int i = 0; i < S64_PER; i++) {
        v[i] = base + i < n ? io[base + i] : 0;
        s += v[i];
    }
    // exclusive scan of the per-thread sums across the block
    const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
    unsigned long long inc = s;
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        unsigned long long t = __shfl_up(inc, d, WAVE);
        if (lane >= d) inc += t;
    }
    if (lane == WAVE - 1) wsum[wid] = inc;
    __syncthreads();
    unsigned long long run = offs[blockIdx.x] + inc - s;
    for (int w = 0; w < wid; w++) run += wsum[w];
#pragma unroll
    for (int i = 0; i < S64_PER; i++) {
        run += v[i];
        if (base + i < n) io[base + i] = run;
    }
}

static int scan_u64_inclusive(unsigned long long *io, uint64_t n, unsigned long long *tmp,
                              hipStream_t s) {
    if (n == 0) return BFC_OK;
    const uint32_t nt = (uint32_t)((n + S64_TILE - 1) / S64_TILE);
    k_s64_tile<<<nt, S64_NT, 0, s>>>(io, n, tmp);
    k_s64_sums<<<1, 64, 0, s>>>(tmp, nt);
    k_s64_apply<<<nt, S64_NT, 0, s>>>(io, n, tmp);
    BFC_HIP(hipGetLastError());
    return BFC_OK;
}

// Draw i: an index below n (uniform) or by weight (prefix sums `pre`, total
// in pre[n-1]); its weight goes to wdraw for the estimate.
__global__ void k_draw(uint64_t k, uint64_t n, uint64_t seed, uint32_t tag,
                       const unsigned long long *pre, const unsigned long long *w,
                       unsigned long long *out, uint32_t *wdraw) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < k;
         i += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t j;
        if (pre) {
            const uint64_t t = draw_below(seed, (uint32_t)i, (uint32_t)(i >> 32), tag, pre[n - 1]);
            uint64_t lo = 0, hi = n;          // first j with pre[j] > t
            while (lo < hi) {
                const uint64_t mid = lo + (hi - lo) / 2;
                if (pre[mid] > t) hi = mid; else lo = mid + 1;
            }
            j = lo;
            wdraw[i] = (uint32_t)w[j];
        } else {
            j = draw_below(seed, (uint32_t)i, (uint32_t)(i >> 32), tag, n);
        }
        out[i] = j;
    }
}

// VSamp: mark the drawn vertices by rank on their side.
__global__ void k_mark_vertices(uint64_t k, const unsigned long long *draw, uint32_t nl,
                                const uint32_t *rank_l, const uint32_t *rank_r, uint8_t *mark_l,
                                uint8_t *mark_r, uint32_t *ids) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < k;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t id = (uint32_t)draw[i];
        ids[i] = id;
        if (id < nl) mark_l[rank_l[id]] = 1;
        else mark_r[rank_r[id - nl]] = 1;
    }
}

__global__ void k_gather_vertex(uint64_t k, const uint32_t *ids, uint32_t nl,
                                const unsigned long long *cl, const unsigned long long *cr,
                                unsigned long long *counts) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < k;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t id = ids[i];
        counts[i] = id < nl ? cl[id] : cr[id - nl];
    }
}

// The draws alone: drawn global ids, each draw's integer weight (1 when
// uniform) and the weight total.
__global__ void k_draw_ids(uint64_t k, uint64_t n, const unsigned long long *draw,
                           const uint32_t *wdraw, const unsigned long long *pre, uint32_t *ids,
                           uint32_t *weights, unsigned long long *total) {
    const uint64_t t0 = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    for (uint64_t i = t0; i < k; i += (uint64_t)gridDim.x * blockDim.x) {
        ids[i] = (uint32_t)draw[i];
        if (weights) weights[i] = pre ? wdraw[i] : 1u;
    }
    if (total && t0 == 0) *total = pre ? pre[n - 1] : n;
}

// ESamp: A-side CSR position of every edge, then mark the drawn edges' starts.
__global__ void k_pos_of_edge(const uint32_t *eidA, uint64_t m, uint32_t *pos) {
    for (uint64_t k = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; k < m;
         k += (uint64_t)gridDim.x * blockDim.x)
        pos[eidA[k]] = (uint32_t)k;
}

__global__ void k_mark_edges(uint64_t k, const unsigned long long *draw, const uint32_t *pos,
                             const uint32_t *offA, uint32_t nA, uint8_t *mark) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < k;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t p = pos[draw[i]];
        uint32_t lo = 0, hi = nA;             // row u with offA[u] <= p < offA[u+1]
        while (lo < hi) {
            const uint32_t mid = lo + (hi - lo) / 2;
            if (offA[mid + 1] > p) hi = mid; else lo = mid + 1;
        }
        mark[lo] = 1;
    }
}

__global__ void k_gather_edge(uint64_t k, const unsigned long long *draw,
                              const unsigned long long *ce, unsigned long long *counts,
                              unsigned long long *eids) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < k;
         i += (uint64_t)gridDim.x * blockDim.x) {
        eids[i] = draw[i];
        counts[i] = ce[draw[i]];
    }
}

// Estimate of a sampler.  Uniform: sum of counts (exact, uint64) * n /
// (4 k).  Weighted: term_i = count_i * (Q / (4 q_i)) summed left to right
// within blocks of COMBINE_BLOCK draws, block sums left to right, over k.
__global__ __launch_bounds__(256) void k_combine(uint64_t k, uint64_t n,
                                                 const unsigned long long *counts,
                                                 const uint32_t *wdraw,
                                                 const unsigned long long *pre,
                                                 double *parts, ProbFlags *f, double *est) {
    __shared__ int ovf;
    if (threadIdx.x == 0) ovf = 0;
    __syncthreads();
    const uint64_t nb = (k + COMBINE_BLOCK - 1) / COMBINE_BLOCK;
    if (pre && !probs_ok(f)) {
        if (threadIdx.x == 0) *est = nan64();
        return;
    }
    if (pre) {
        const double Q = (double)pre[n - 1];
        for (uint64_t b = threadIdx.x; b < nb; b += blockDim.x) {
            double part = 0.0;
            const uint64_t e = min((uint64_t)(b + 1) * COMBINE_BLOCK, k);
            for (uint64_t i = b * COMBINE_BLOCK; i < e; i++)
                part += (double)counts[i] * (Q / (4.0 * (double)wdraw[i]));
            parts[b] = part;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double total = 0.0;
            for (uint64_t b = 0; b < nb; b++) total += parts[b];
            *est = total / (double)k;
        }
    } else {
        // exact uint64 sums per thread, then in thread order
        unsigned long long s = 0;
        for (uint64_t i = threadIdx.x; i < k; i += blockDim.x) {
            const unsigned long long c = counts[i];
            if (s + c < s) ovf = 1;
            s += c;
        }
        ((unsigned long long *)parts)[threadIdx.x] = s;
        __syncthreads();
        if (threadIdx.x == 0) {
            unsigned long long t = 0;
            for (unsigned i = 0; i < blockDim.x; i++) {
                const unsigned long long c = ((unsigned long long *)parts)[i];
                if (t + c < t) ovf = 1;
                t += c;
            }
            *est = ovf ? nan64() : ((double)t * (double)n) / (4.0 * (double)k);
            if (ovf) f->overflow = 1;
        }
    }
}

// ------------------------------------------------------------------ Fast-eBFC
// ESamp with Fast-eBFC (Sec. 5.5): each drawn edge e = (a, x) gets alpha
// trials; a trial picks b among the neighbours of x and y among those of a
// and hits iff b != a, y != x and (b, y) is an edge.  hits * d_a * d_x has
// mean B_e.
struct FastArgs {
    const uint32_t *off_l, *adj_l, *off_r, *adj_r;
    const uint32_t *ea, *ex;        // per draw: L rank and R rank of the edge
    uint64_t k, seed;
    uint32_t alpha;
};

// Per draw: the drawn edge's endpoints as ranks (pos = L-side CSR position
// of every input edge); clears the hit counter and reports the edge index.
__global__ void k_fast_setup(uint64_t k, const unsigned long long *draw, const uint32_t *pos,
                             const uint32_t *off_l, uint32_t nl, const uint32_t *adj_l,
                             uint32_t *ea, uint32_t *ex, uint32_t *hits,
                             unsigned long long *eids) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < k;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t p = pos[draw[i]];
        uint32_t lo = 0, hi = nl;             // row a with off_l[a] <= p < off_l[a+1]
        while (lo < hi) {
            const uint32_t mid = lo + (hi - lo) / 2;
            if (off_l[mid + 1] > p) hi = mid; else lo = mid + 1;
        }
        ea[i] = lo;
        ex[i] = adj_l[p];
        hits[i] = 0;
        eids[i] = draw[i];
    }
}

// One trial's probe: lower bound of `target` in row[lo..hi), with `found`
// set when a probe equals it (the lower bound is always probed before the
// search ends, so no final load is needed).  Lanes without a probe (a miss
// already decided, or no trial) get an empty search.
struct Probe {
    const uint32_t *row;
    uint32_t lo, hi, target;
    bool found;
};

__device__ inline Probe trial_probe(const FastArgs &f, uint64_t i, uint32_t j, bool valid) {
    Probe t = {f.adj_l, 0, 0, 0, false};
    if (!valid) return t;
    const uint32_t a = f.ea[i], x = f.ex[i];
    const uint32_t la = f.off_l[a], da = f.off_l[a + 1] - la;
    const uint32_t lx = f.off_r[x], dx = f.off_r[x + 1] - lx;
    const uint64_t rx = (0 - (uint64_t)dx) % dx, ra = (0 - (uint64_t)da) % da;
    uint32_t o[4];
    uint64_t x1, x2;
    for (uint32_t attempt = 0;; attempt++) {
        philox((uint32_t)i, j, TAG_FAST, attempt, f.seed, o);
        x1 = (uint64_t)o[0] | ((uint64_t)o[1] << 32);
        x2 = (uint64_t)o[2] | ((uint64_t)o[3] << 32);
        if ((rx == 0 || x1 < 0 - rx) && (ra == 0 || x2 < 0 - ra)) break;
    }
    const uint32_t b = f.adj_r[lx + (uint32_t)(x1 % dx)];   // L rank
    const uint32_t y = f.adj_l[la + (uint32_t)(x2 % da)];   // R rank
    if (b != a && y != x) {
        const uint32_t lb = f.off_l[b], db = f.off_l[b + 1] - lb;
        const uint32_t ly = f.off_r[y], dy = f.off_r[y + 1] - ly;
        if (db <= dy) {
            t.row = f.adj_l + lb;
            t.hi = db;
            t.target = y;
        } else {
            t.row = f.adj_r + ly;
            t.hi = dy;
            t.target = b;
        }
    }
    return t;
}

// One wave per unit (draw, 64 consecutive trials), one trial per lane; a
// wave adds its hits to the draw's counter with one atomic.  Every probe
// index lies in [lo, hi), inside the probed row.  Running two or four units
// side by side per wave was slower: a wave's searches diverge, and the
// merged loop runs as long as the longest of them.
__global__ __launch_bounds__(256) void k_fast_trials(FastArgs f, uint32_t *hits) {
    const uint32_t lane = threadIdx.x & (WAVE - 1);
    const uint64_t nchunk = (f.alpha + WAVE - 1) / WAVE;
    const uint64_t units = f.k * nchunk;
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) / WAVE;
    for (uint64_t u = (blockIdx.x * (uint64_t)blockDim.x + threadIdx.x) / WAVE; u < units;
         u += nwaves) {
        const uint64_t i = u / nchunk;
        const uint32_t j = (uint32_t)(u - i * nchunk) * WAVE + lane;
        Probe t = trial_probe(f, i, j, j < f.alpha);
        while (t.lo < t.hi) {
            const uint32_t mid = (t.lo + t.hi) >> 1;
            const uint32_t v = t.row[mid];
            if (v < t.target) {
                t.lo = mid + 1;
            } else {
                t.hi = mid;
                t.found |= v == t.target;
            }
        }
        const uint64_t mask = __ballot(t.found);
        if (lane == 0 && mask) atomicAdd(&hits[i], (uint32_t)__popcll(mask));
    }
}

// Estimate: term_i = ((double)hits_i * (double)(d_a d_x)) * s_i with s_i =
// m / 4 (uniform) or Q / (4 q_i) (weighted), summed left to right within
// blocks of COMBINE_BLOCK draws, block sums left to right, over k * alpha.
// The terms are formed in parallel, each block's sum by one thread, the
// total by one thread: the same additions in the same order.
__global__ void k_fast_terms(FastArgs f, uint64_t m, const uint32_t *hits, const uint32_t *wdraw,
                             const unsigned long long *pre, double *terms) {
    const double su = (double)m / 4.0;
    const double Q = pre ? (double)pre[m - 1] : 0.0;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < f.k;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t a = f.ea[i], x = f.ex[i];
        const uint64_t dd = (uint64_t)(f.off_l[a + 1] - f.off_l[a]) *
                            (f.off_r[x + 1] - f.off_r[x]);
        const double sc = pre ? Q / (4.0 * (double)wdraw[i]) : su;
        terms[i] = ((double)hits[i] * (double)dd) * sc;
    }
}

__global__ void k_block_sums(const double *terms, uint64_t k, double *parts) {
    const uint64_t nb = (k + COMBINE_BLOCK - 1) / COMBINE_BLOCK;
    for (uint64_t b = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; b < nb;
         b += (uint64_t)gridDim.x * blockDim.x) {
        double part = 0.0;
        const uint64_t e = min((uint64_t)(b + 1) * COMBINE_BLOCK, k);
        for (uint64_t i = b * COMBINE_BLOCK; i < e; i++) part += terms[i];
        parts[b] = part;
    }
}

__global__ void k_fast_total(uint64_t k, uint32_t alpha, const double *parts, const ProbFlags *f,
                             double *est) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const uint64_t nb = (k + COMBINE_BLOCK - 1) / COMBINE_BLOCK;
        double total = 0.0;
        for (uint64_t b = 0; b < nb; b++) total += parts[b];
        *est = (f && !probs_ok(f)) ? nan64() : total / ((double)k * (double)alpha);
    }
}

// ------------------------------------------------------------------ WSamp
// WSamp (Sec. 5.3).  Wedges are numbered 0 .. W-1: vertices in global order
// (L ids, then n_left + R id) own consecutive ranges of C(d,2) numbers, and
// number p inside u's range is the pair of neighbour positions (j1, j2),
// j1 < j2, with p = C(j2,2) + j1 (neighbours in ascending rank order).  A
// uniform number is a uniform wedge; its butterflies are |G_v n G_w| - 1.
__device__ inline uint64_t choose2_u64(uint64_t d) { return d < 2 ? 0 : d * (d - 1) / 2; }

__global__ void k_wedge_weights(uint32_t nl, uint32_t nr, const uint32_t *rank_l,
                                const uint32_t *rank_r, const uint32_t *off_l,
                                const uint32_t *off_r, unsigned long long *pre) {
    const uint64_t n = (uint64_t)nl + nr;
    for (uint64_t v = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; v < n;
         v += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t d;
        if (v < nl) {
            const uint32_t rk = rank_l[v];
            d = off_l[rk + 1] - off_l[rk];
        } else {
            const uint32_t rk = rank_r[v - nl];
            d = off_r[rk + 1] - off_r[rk];
        }
        pre[v] = choose2_u64(d);
    }
}

// First index v < n with pre[v] > t (n if none), pre non-decreasing, found
// by the whole wave: each step the 64 lanes read 64 evenly spaced entries
// of the remaining range and a ballot keeps the segment holding the
// answer, so about log64(n) dependent reads instead of log2(n).  Every lane
// returns the same index.
__device__ inline uint64_t wave_first_above(const unsigned long long *pre, uint64_t n, uint64_t t,
                                            uint32_t lane) {
    uint64_t lo = 0, hi = n;            // answer in [lo, hi]; hi == n or pre[hi] > t
    while (hi - lo > WAVE) {
        const uint64_t step = (hi - lo + WAVE - 1) / WAVE;
        const uint64_t e = lo + (uint64_t)(lane + 1) * step;
        const uint64_t p = (e < hi ? e : hi) - 1;   // probe of this lane, in [lo, hi)
        const uint64_t mask = __ballot(pre[p] > t);
        if (!mask) {
            lo = hi;                    // every probe, the last one included, is <= t
        } else {
            const uint32_t f = (uint32_t)__ffsll((unsigned long long)mask) - 1;
            const uint64_t ef = lo + (uint64_t)(f + 1) * step;
            const uint64_t pf = (ef < hi ? ef : hi) - 1;
            const uint64_t nlo = f ? lo + (uint64_t)f * step : lo;   // one past probe f - 1
            lo = nlo < pf ? nlo : pf;
            hi = pf;
        }
    }
    const uint64_t q = lo + lane;
    const uint64_t mask = __ballot(q < hi && pre[q] > t);
    return mask ? lo + (uint64_t)__ffsll((unsigned long long)mask) - 1 : hi;
}

struct WsampArgs {
    const uint32_t *off_l, *adj_l, *off_r, *adj_r, *rank_l, *rank_r, *id_l, *id_r;
    const unsigned long long *pre;      // inclusive prefix sums of C(d,2), global order
    uint64_t n, W, k, seed;
    uint32_t nl;
};

// One wave per draw: every lane decodes the same wedge; the shorter
// endpoint list is spread over the lanes and each entry is searched in the
// longer one.
__global__ __launch_bounds__(256) void k_wsamp(WsampArgs a, uint32_t *mids, uint32_t *ends,
                                               unsigned long long *counts) {
    const uint32_t lane = threadIdx.x & (WAVE - 1);
    const uint64_t nwaves = ((uint64_t)gridDim.x * blockDim.x) / WAVE;
    for (uint64_t i = (blockIdx.x * (uint64_t)blockDim.x + threadIdx.x) / WAVE; i < a.k;
         i += nwaves) {
        const uint64_t t = draw_below(a.seed, (uint32_t)i, (uint32_t)(i >> 32), TAG_WDRAW, a.W);
        const uint64_t u = wave_first_above(a.pre, a.n, t, lane);
        if (u >= a.n) {                       // totals disagree: report nothing, read nothing
            if (lane == 0) {
                mids[i] = 0xFFFFFFFFu;
                ends[2 * i] = ends[2 * i + 1] = 0xFFFFFFFFu;
                counts[i] = 0;
            }
            continue;
        }
        const uint64_t p = t - (u ? a.pre[u - 1] : 0);
        // j2 = the largest j with C(j,2) <= p (a floating-point guess, then exact fixes)
        uint64_t j2 = (uint64_t)((1.0 + sqrt(1.0 + 8.0 * (double)p)) * 0.5);
        while (j2 > 1 && choose2_u64(j2) > p) j2--;
        while (choose2_u64(j2 + 1) <= p) j2++;
        const uint64_t j1 = p - choose2_u64(j2);
        const uint32_t *offB, *adjB;          // rows of the endpoints' side
        uint32_t v, w, e1, e2;
        if (u < a.nl) {
            const uint32_t base = a.off_l[a.rank_l[u]];
            v = a.adj_l[base + j1];
            w = a.adj_l[base + j2];
            e1 = a.nl + a.id_r[v];
            e2 = a.nl + a.id_r[w];
            offB = a.off_r;
            adjB = a.adj_r;
        } else {
            const uint32_t base = a.off_r[a.rank_r[u - a.nl]];
            v = a.adj_r[base + j1];
            w = a.adj_r[base + j2];
            e1 = a.id_l[v];
            e2 = a.id_l[w];
            offB = a.off_l;
            adjB = a.adj_l;
        }
        const uint32_t lv = offB[v], dv = offB[v + 1] - lv;
        const uint32_t lw = offB[w], dw = offB[w + 1] - lw;
        const uint32_t ls = dv <= dw ? lv : lw, ds = dv <= dw ? dv : dw;
        const uint32_t lb = dv <= dw ? lw : lv, db = dv <= dw ? dw : dv;
        uint64_t c = 0;
        for (uint32_t b0 = 0; b0 < ds; b0 += WAVE) {
            const uint32_t idx = b0 + lane;
            bool found = false;
            if (idx < ds) {
                const uint32_t target = adjB[ls + idx], *row = adjB + lb;
                uint32_t lo = 0, hi = db;     // lower bound, found when probed equal
                while (lo < hi) {
                    const uint32_t mid = (lo + hi) >> 1;
                    const uint32_t v = row[mid];
                    if (v < target) {
                        lo = mid + 1;
                    } else {
                        hi = mid;
                        found |= v == target;
                    }
                }
            }
            c += (uint64_t)__popcll(__ballot(found));
        }
        if (lane == 0) {
            mids[i] = (uint32_t)u;
            ends[2 * i] = e1;
            ends[2 * i + 1] = e2;
            counts[i] = c - 1;                // the midpoint itself is common
        }
    }
}

// Estimate: ((double)sum counts * (double)W) / (4 k), the sum exact in uint64
// (integer additions: any order gives the same sum).
__global__ void k_zero_u64(unsigned long long *p) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *p = 0;
}

__global__ __launch_bounds__(256) void k_wsamp_sum(uint64_t k, const unsigned long long *counts,
                                                   unsigned long long *acc) {
    __shared__ unsigned long long red[256 / WAVE];
    unsigned long long s = 0;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < k;
         i += (uint64_t)gridDim.x * blockDim.x)
        s += counts[i];
    s = block_sum64<256>(s, red);
    if (threadIdx.x == 0 && s) atomicAdd(acc, s);
}

__global__ void k_wsamp_est(uint64_t k, double W, const unsigned long long *acc, double *est) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *est = ((double)*acc * W) / (4.0 * (double)k);
}

// ------------------------------------------------------------------ (eps, delta)
// Median of means: group q holds x[q r .. q r + r), its mean sums left to
// right and divides by r; the median is the mean of sorted position
// (g - 1) / 2, ties broken by group index.
constexpr uint32_t MOM_MAX_GROUPS = 4096;

__global__ __launch_bounds__(256) void k_median_of_means(const double *x, uint32_t g, uint32_t r,
                                                         double *means, double *median) {
    for (uint32_t q = threadIdx.x; q < g; q += blockDim.x) {
        double s = 0.0;
        for (uint32_t i = 0; i < r; i++) s += x[(uint64_t)q * r + i];
        means[q] = s / (double)r;
    }
    __syncthreads();
    const uint32_t mid = (g - 1) / 2;
    for (uint32_t q = threadIdx.x; q < g; q += blockDim.x) {
        const double mq = means[q];
        uint32_t rank = 0;
        for (uint32_t j = 0; j < g; j++) {
            const double mj = means[j];
            rank += (mj < mq) || (mj == mq && j < q);
        }
        if (rank == mid) *median = mq;
    }
}

static inline unsigned grid_for(uint64_t n, int nt = 256) {
    uint64_t g = (n + nt - 1) / nt;
    if (g < 1) g = 1;
    if (g > 65535ull * 16) g = 65535ull * 16;
    return (unsigned)g;
}

// ------------------------------------------------------------------ host: sparsifiers
static inline unsigned rows_grid(uint32_t n) {
    unsigned g = grid_for(n, 4);
    return g > 8192 ? 8192 : g;
}

static void side_views(const bfc_graph *g, SideView &L, SideView &R) {
    L = SideView{g->off_l, g->adj_l, g->xpos_l, g->id_l, g->id_r, g->n_left, 0};
    R = SideView{g->off_r, g->adj_r, g->xpos_r, g->id_r, g->id_l, g->n_right, 1};
}

static KeepRule espar_rule(double p, uint64_t seed) {
    KeepRule k = {};
    k.kind = 0;
    k.seed = seed;
    k.keep_all = p >= 1.0;
    k.thresh = k.keep_all ? 0 : (uint64_t)ldexp(p, 64);
    return k;
}

// ClrSpar's rule; the colours of both sides go to col_l / col_r.
static int clrspar_rule(const bfc_graph *g, uint32_t ncolors, uint64_t seed, uint32_t *col_l,
                        uint32_t *col_r, KeepRule &k, hipStream_t s) {
    k = KeepRule{};
    k.kind = 1;
    k.seed = seed;
    k.keep_all = ncolors == 1;
    k.col_l = col_l;
    k.col_r = col_r;
    if (!k.keep_all) {
        if (g->n_left)
            k_colours<<<grid_for(g->n_left), 256, 0, s>>>(g->n_left, 0, ncolors, seed, g->id_l,
                                                          col_l);
        if (g->n_right)
            k_colours<<<grid_for(g->n_right), 256, 0, s>>>(g->n_right, 1, ncolors, seed, g->id_r,
                                                           col_r);
        BFC_HIP(hipGetLastError());
    }
    return BFC_OK;
}

static int rule_of(const bfc_graph *g, const bfc_replica &r, uint32_t *col_l, uint32_t *col_r,
                   KeepRule &k, hipStream_t s) {
    if (r.kind == BFC_REPLICA_ESPAR) {
        k = espar_rule(r.p, r.seed);
        return BFC_OK;
    }
    return clrspar_rule(g, r.ncolors, r.seed, col_l, col_r, k, s);
}

// Buffers of one replica's keep flags: flags in both CSR orders (scanned in
// place), kept-vertex marks of both sides (scanned in place), colours, and
// the row of every CSR position (filled once per call by keep_rows).
struct KeepWs {
    uint32_t *fl, *fr, *ml, *mr, *scan_tmp, *col_l, *col_r, *row_l, *row_r;
};

static void carve_keep(Carver &c, const bfc_graph *g, KeepWs &w) {
    const uint64_t m = g->n_edges;
    uint64_t big = m;
    if (g->n_left > big) big = g->n_left;
    if (g->n_right > big) big = g->n_right;
    w.fl = c.take<uint32_t>(pad64(m));
    w.fr = c.take<uint32_t>(pad64(m));
    w.ml = c.take<uint32_t>(pad64(g->n_left));
    w.mr = c.take<uint32_t>(pad64(g->n_right));
    w.scan_tmp = c.take<uint32_t>(scan_tmp_elems(big));
    w.col_l = c.take<uint32_t>(pad64(g->n_left));
    w.col_r = c.take<uint32_t>(pad64(g->n_right));
    w.row_l = c.take<uint32_t>(pad64(m));
    w.row_r = c.take<uint32_t>(pad64(m));
}

static int keep_rows(const bfc_graph *g, KeepWs &w, hipStream_t s) {
    if (!g->n_edges) return BFC_OK;
    k_row_of<<<rows_grid(g->n_left), 256, 0, s>>>(g->off_l, g->n_left, w.row_l);
    k_row_of<<<rows_grid(g->n_right), 256, 0, s>>>(g->off_r, g->n_right, w.row_r);
    BFC_HIP(hipGetLastError());
    return BFC_OK;
}

// Offsets and entries of one side's kept rows (EmitArgs above).
static int emit(const EmitArgs &a, uint64_t m, hipStream_t s) {
    k_emit_offsets<<<grid_for(a.n), 256, 0, s>>>(a);
    k_emit_entries<<<grid_for(m), 256, 0, s>>>(a, m);
    BFC_HIP(hipGetLastError());
    return BFC_OK;
}

// Keep flags of both CSR orders and their inclusive scans; with `marks`,
// the kept-vertex marks of both sides and their inclusive scans too.
static int keep_and_scan(const bfc_graph *g, const KeepRule &k, KeepWs &w, bool marks,
                         hipStream_t s) {
    SideView L, R;
    side_views(g, L, R);
    const uint64_t m = g->n_edges;
    if (m) {
        k_keep_flags<<<grid_for(m), 256, 0, s>>>(L, k, w.row_l, m, w.fl);
        k_keep_flags<<<grid_for(m), 256, 0, s>>>(R, k, w.row_r, m, w.fr);
        BFC_HIP(hipGetLastError());
        BFC_TRY(scan_u32_inclusive(w.fl, w.fl, m, w.scan_tmp, s));
        BFC_TRY(scan_u32_inclusive(w.fr, w.fr, m, w.scan_tmp, s));
    }
    if (marks) {
        if (g->n_left) {
            k_kept_marks<<<grid_for(g->n_left), 256, 0, s>>>(g->off_l, g->n_left, w.fl, w.ml);
            BFC_TRY(scan_u32_inclusive(w.ml, w.ml, g->n_left, w.scan_tmp, s));
        }
        if (g->n_right) {
            k_kept_marks<<<grid_for(g->n_right), 256, 0, s>>>(g->off_r, g->n_right, w.fr, w.mr);
            BFC_TRY(scan_u32_inclusive(w.mr, w.mr, g->n_right, w.scan_tmp, s));
        }
        BFC_HIP(hipGetLastError());
    }
    return BFC_OK;
}

// The single sparsifier calls: the kept graph laid out on the graph's own
// sizes (rows beyond the kept vertices empty), counted from the side
// ExactBFC's rule picks for the graph itself.  The count is the same from
// either side; the kept sizes never leave the device, so the call is
// asynchronous.
struct SparWs {
    KeepWs k;
    uint32_t *off_l, *adj_l, *off_r, *adj_r, *xpos;
    void *work;                 // the exact count's workspace
    size_t work_bytes;
};

static void carve_spar(Carver &c, const bfc_graph *g, SparWs &w) {
    carve_keep(c, g, w.k);
    const uint64_t m = g->n_edges;
    w.off_l = c.take<uint32_t>(pad64((uint64_t)g->n_left + 1));
    w.off_r = c.take<uint32_t>(pad64((uint64_t)g->n_right + 1));
    w.adj_l = c.take<uint32_t>(pad64(m + ADJ_SLACK));
    w.adj_r = c.take<uint32_t>(pad64(m + ADJ_SLACK));
    w.xpos = c.take<uint32_t>(pad64(m));
    w.work_bytes = exact_ws_bound(g->n_left, g->n_right, m);
    w.work = c.take<char>(w.work_bytes);
}

static int sparsify_count(const bfc_graph *g, const KeepRule &k, SparWs &w, uint64_t *d_beta,
                          uint64_t *d_kept, hipStream_t s) {
    const uint64_t m = g->n_edges;
    const uint32_t nl = g->n_left, nr = g->n_right;
    BFC_TRY(keep_rows(g, w.k, s));
    BFC_TRY(keep_and_scan(g, k, w.k, true, s));
    const int side = bfc_side_used(g, BFC_SIDE_AUTO);
    if (side < 0) return side;
    const bool from_r = side == BFC_SIDE_R;
    if (m) {
        EmitArgs el = {g->off_l, g->adj_l, g->xpos_l, w.k.fl, w.k.fr, w.k.ml, w.k.mr, nl,
                       0, 0, 0, w.off_l, w.adj_l, from_r ? nullptr : w.xpos, nullptr};
        EmitArgs er = {g->off_r, g->adj_r, g->xpos_r, w.k.fr, w.k.fl, w.k.mr, w.k.ml, nr,
                       0, 0, 0, w.off_r, w.adj_r, from_r ? w.xpos : nullptr, nullptr};
        BFC_TRY(emit(el, m, s));
        BFC_TRY(emit(er, m, s));
    }
    k_kept_tail<<<grid_for(m > nl ? m : (uint64_t)nl + 1), 256, 0, s>>>(w.off_l, nl, w.k.ml,
                                                                        w.k.fl, m, w.adj_l);
    k_kept_tail<<<grid_for(m > nr ? m : (uint64_t)nr + 1), 256, 0, s>>>(w.off_r, nr, w.k.mr,
                                                                        w.k.fr, m, w.adj_r);
    if (d_kept) k_kept_total<<<1, 64, 0, s>>>(w.k.fl, m, (unsigned long long *)d_kept);
    BFC_HIP(hipGetLastError());
    // the kept graph: the graph's sizes and statistics as upper bounds
    bfc_graph h = *g;
    h.off_l = w.off_l; h.adj_l = w.adj_l; h.off_r = w.off_r; h.adj_r = w.adj_r;
    h.xpos_l = from_r ? nullptr : w.xpos;
    h.xpos_r = from_r ? w.xpos : nullptr;
    h.eid_l = h.eid_r = h.rank_l = h.rank_r = h.id_l = h.id_r = nullptr;
    return bfc_exact(&h, side, d_beta, w.work, w.work_bytes, s);
}

}  // namespace bfc

using namespace bfc;

extern "C" {

int bfc_spar_ws_size(const bfc_graph *g, size_t *bytes) {
    if (!g || !bytes) return BFC_E_NULL;
    Carver c(nullptr, 0);
    SparWs w;
    carve_spar(c, g, w);
    *bytes = c.used;
    return BFC_OK;
}

static int spar_args(const bfc_graph *g, uint64_t *d_beta, double *d_est, uint64_t *d_kept,
                     void *d_ws) {
    if (!g || !d_beta || !d_est || !d_ws) return BFC_E_NULL;
    if (!aligned256(d_ws) || ((uintptr_t)d_beta & 7) || ((uintptr_t)d_est & 7) ||
        ((uintptr_t)d_kept & 7))
        return BFC_E_ALIGN;
    return BFC_OK;
}

int bfc_espar(const bfc_graph *g, double p, uint64_t seed, uint64_t *d_beta, double *d_est,
              uint64_t *d_kept, void *d_ws, size_t ws_bytes, hipStream_t s) {
    BFC_TRY(spar_args(g, d_beta, d_est, d_kept, d_ws));
    if (!(p > 0.0) || !(p <= 1.0)) return BFC_E_ARG;
    Carver c(d_ws, ws_bytes);
    SparWs w;
    carve_spar(c, g, w);
    if (!c.fits()) return BFC_E_WS_SMALL;
    BFC_TRY(sparsify_count(g, espar_rule(p, seed), w, d_beta, d_kept, s));
    k_est_scale<<<1, 64, 0, s>>>((unsigned long long *)d_beta, (p * p) * (p * p), 0.0, d_est);
    BFC_HIP(hipGetLastError());
    return BFC_OK;
}

int bfc_clrspar(const bfc_graph *g, uint32_t ncolors, uint64_t seed, uint64_t *d_beta,
                double *d_est, uint64_t *d_kept, void *d_ws, size_t ws_bytes, hipStream_t s) {
    BFC_TRY(spar_args(g, d_beta, d_est, d_kept, d_ws));
    if (ncolors == 0) return BFC_E_ARG;
    Carver c(d_ws, ws_bytes);
    SparWs w;
    carve_spar(c, g, w);
    if (!c.fits()) return BFC_E_WS_SMALL;
    KeepRule k;
    BFC_TRY(clrspar_rule(g, ncolors, seed, w.k.col_l, w.k.col_r, k, s));
    BFC_TRY(sparsify_count(g, k, w, d_beta, d_kept, s));
    const double N = (double)ncolors;
    k_est_scale<<<1, 64, 0, s>>>((unsigned long long *)d_beta, 0.0, N * N * N, d_est);
    BFC_HIP(hipGetLastError());
    return BFC_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ host: replica batches
// Many ESpar / ClrSpar replicas of one graph counted together.  Phase 1
// measures each replica's kept graph (edges, vertices keeping an edge, sums
// of squared kept degrees).  Phase 2 builds every kept graph, oriented by
// ExactBFC's rule on its own degrees, as one part of a disjoint union laid
// out from those sizes (part i's union L ranks start at VL_i, its R ranks at
// VR_i, its edges at E_i), and bfc_exact_parts counts all parts in one plan
// and one launch per kernel class.  Phase 2 only launches kernels, so it can
// be captured into a HIP graph and replayed.  Every replica's count and
// estimate equal those of bfc_espar / bfc_clrspar with the same parameters
// and seed.
namespace bfc {

// Replica i's kept sizes against the ones phase 2 was laid out for.
__global__ void k_check_part(const uint32_t *fl, uint64_t m, const uint32_t *ml, uint32_t nl,
                             const uint32_t *mr, uint32_t nr, uint64_t kept, uint32_t kl,
                             uint32_t kr, uint32_t *bad) {
    if (threadIdx.x || blockIdx.x) return;
    const uint64_t k = m ? fl[m - 1] : 0u;
    const uint32_t a = nl ? ml[nl - 1] : 0u, b = nr ? mr[nr - 1] : 0u;
    if (k != kept || a != kl || b != kr) atomicOr(bad, 1u);
}

// Per-part values: the part's first union L rank, the divisor / multiplier
// of its estimate.
__global__ void k_part_meta(uint32_t i, uint32_t vbase, double div, double mul, uint32_t *part_l,
                            double *d_div, double *d_mul) {
    if (threadIdx.x || blockIdx.x) return;
    part_l[i] = vbase;
    d_div[i] = div;
    d_mul[i] = mul;
}

// Ends of the union's offset arrays.  A batch with a part that did not match
// its sizes becomes a graph without edges (every row empty), so the count
// reads only valid memory; its results are then marked as invalid.
__global__ void k_union_finish(uint32_t *off_l, uint32_t nl, uint32_t *off_r, uint32_t nr,
                               uint32_t M, uint32_t *part_l, uint32_t nparts, const uint32_t *bad) {
    const bool b = *bad != 0u;
    const uint64_t lim = (uint64_t)(nl > nr ? nl : nr) + 1;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < lim;
         i += (uint64_t)gridDim.x * blockDim.x) {
        if (i == 0) {
            off_l[nl] = b ? 0u : M;
            off_r[nr] = b ? 0u : M;
            part_l[nparts] = nl;
        }
        if (b && i < nl) off_l[i] = 0u;
        if (b && i < nr) off_r[i] = 0u;
    }
}

// Estimates in the single-replica expressions; an invalid batch (sizes not
// those of phase 1) gets counts 2^64 - 1 and NaN estimates.
__global__ void k_est_batch(unsigned long long *beta, const double *div, const double *mul,
                            uint32_t n, const uint32_t *bad, double *est) {
    const bool b = *bad != 0u;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        if (b) {
            beta[i] = ~0ull;
            est[i] = __longlong_as_double(0x7FF8000000000000ll);
            continue;
        }
        const double x = (double)beta[i];
        est[i] = div[i] != 0.0 ? x / div[i] : x * mul[i];
    }
}

__global__ void k_zero_u32x(uint32_t *p, uint64_t n) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

__global__ void k_zero_u64x(unsigned long long *p, uint64_t n) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

static int check_replicas(uint32_t nrep, const bfc_replica *reps) {
    if (!reps) return BFC_E_NULL;
    if (nrep == 0) return BFC_E_ARG;
    for (uint32_t i = 0; i < nrep; i++) {
        const bfc_replica &r = reps[i];
        if (r.kind == BFC_REPLICA_ESPAR) {
            if (!(r.p > 0.0) || !(r.p <= 1.0)) return BFC_E_ARG;
        } else if (r.kind == BFC_REPLICA_CLRSPAR) {
            if (r.ncolors == 0) return BFC_E_ARG;
        } else {
            return BFC_E_ARG;
        }
    }
    return BFC_OK;
}

// The union's layout from phase 1: part i starts from R (its sides
// exchanged) when its sum of squared kept L degrees is below its R one.
struct UnionLayout {
    std::vector<uint64_t> ebase;
    std::vector<uint32_t> vl, vr;       // first union L / R rank of each part
    std::vector<uint8_t> swapped;
    uint64_t M, NL, NR, wedges;         // wedges: sum over union R vertices of C(d, 2)
};

static int union_layout(uint32_t nrep, const bfc_replica_info *info, UnionLayout &u) {
    u.ebase.assign(nrep + 1, 0);
    u.vl.assign(nrep + 1, 0);
    u.vr.assign(nrep + 1, 0);
    u.swapped.assign(nrep, 0);
    uint64_t M = 0, NL = 0, NR = 0, W = 0;
    for (uint32_t i = 0; i < nrep; i++) {
        const bfc_replica_info &r = info[i];
        const bool sw = r.sumsq_left < r.sumsq_right;
        u.swapped[i] = sw;
        u.ebase[i] = M;
        u.vl[i] = (uint32_t)NL;
        u.vr[i] = (uint32_t)NR;
        M += r.kept;
        NL += sw ? r.n_right : r.n_left;
        NR += sw ? r.n_left : r.n_right;
        // midpoints are the part's other side: sum C(d,2) = (sum d^2 - sum d) / 2
        const uint64_t sq = sw ? r.sumsq_left : r.sumsq_right;
        if (sq < r.kept) return BFC_E_ARG;
        W += (sq - r.kept) / 2;
        if (M > 0xFFFFFFFFull - ADJ_SLACK || NL > 0xFFFFFFFEull || NR > 0xFFFFFFFEull)
            return BFC_E_TOO_LARGE;
    }
    u.ebase[nrep] = M;
    u.vl[nrep] = (uint32_t)NL;
    u.vr[nrep] = (uint32_t)NR;
    u.M = M;
    u.NL = NL;
    u.NR = NR;
    u.wedges = W;
    return BFC_OK;
}

// The union as a bfc_graph (L = every part's start side).  Ranks are the
// union's vertex numbers (rank_l left NULL: the identity for the per-part
// sums); the largest degree of the graph bounds every kept degree.
static bfc_graph union_graph(const bfc_graph *g, const UnionLayout &u, uint32_t *off_l,
                             uint32_t *adj_l, uint32_t *xpos_l, uint32_t *off_r, uint32_t *adj_r) {
    bfc_graph h = {};
    h.n_left = (uint32_t)u.NL;
    h.n_right = (uint32_t)u.NR;
    h.n_edges = u.M;
    h.off_l = off_l; h.adj_l = adj_l; h.xpos_l = xpos_l;
    h.off_r = off_r; h.adj_r = adj_r;
    const uint32_t md = g->max_deg_l > g->max_deg_r ? g->max_deg_l : g->max_deg_r;
    h.max_deg_l = h.max_deg_r = md;
    h.wedges_mid_r = u.wedges;
    h.sumsq_l = 1;                       // the union is always counted from L
    h.device = g->device;
    return h;
}

struct BatchWs {
    KeepWs k;
    uint32_t *off_l, *adj_l, *xpos_l, *off_r, *adj_r, *part_l, *bad;
    double *div, *mul;
    void *work;                          // bfc_exact_parts on the union
    size_t work_bytes;
};

static int carve_batch(Carver &c, const bfc_graph *g, uint32_t nrep, const bfc_replica_info *info,
                       BatchWs &w, UnionLayout &u) {
    BFC_TRY(union_layout(nrep, info, u));
    carve_keep(c, g, w.k);
    w.off_l = c.take<uint32_t>(pad64(u.NL + 1));
    w.off_r = c.take<uint32_t>(pad64(u.NR + 1));
    w.adj_l = c.take<uint32_t>(pad64(u.M + ADJ_SLACK));
    w.adj_r = c.take<uint32_t>(pad64(u.M + ADJ_SLACK));
    w.xpos_l = c.take<uint32_t>(pad64(u.M));
    w.part_l = c.take<uint32_t>(nrep + 1);
    w.bad = c.take<uint32_t>(1);
    w.div = c.take<double>(nrep);
    w.mul = c.take<double>(nrep);
    bfc_graph h = union_graph(g, u, nullptr, nullptr, nullptr, nullptr, nullptr);
    size_t pb = 0;
    BFC_TRY(bfc_exact_parts_ws_size(&h, &pb));
    w.work_bytes = pb;
    w.work = c.take<char>(pb);
    return BFC_OK;
}

}  // namespace bfc

extern "C" {

int bfc_spar_batch_filter_ws_size(const bfc_graph *g, uint32_t nrep, size_t *bytes) {
    if (!g || !bytes) return BFC_E_NULL;
    Carver c(nullptr, 0);
    KeepWs w;
    carve_keep(c, g, w);
    c.take<unsigned long long>(5 * (uint64_t)nrep);
    *bytes = c.used;
    return BFC_OK;
}

int bfc_spar_batch_filter(const bfc_graph *g, uint32_t nrep, const bfc_replica *reps,
                          bfc_replica_info *h_info, void *d_ws, size_t ws_bytes, hipStream_t s) {
    if (!g || !h_info || !d_ws) return BFC_E_NULL;
    BFC_TRY(check_replicas(nrep, reps));
    if (!aligned256(d_ws)) return BFC_E_ALIGN;
    Carver c(d_ws, ws_bytes);
    KeepWs w;
    carve_keep(c, g, w);
    unsigned long long *st = c.take<unsigned long long>(5 * (uint64_t)nrep);
    if (!c.fits()) return BFC_E_WS_SMALL;
    k_zero_u64x<<<grid_for(5 * (uint64_t)nrep), 256, 0, s>>>(st, 5 * (uint64_t)nrep);
    BFC_TRY(keep_rows(g, w, s));
    unsigned gl = grid_for(g->n_left), gr = grid_for(g->n_right);
    if (gl > 4096) gl = 4096;
    if (gr > 4096) gr = 4096;
    for (uint32_t i = 0; i < nrep; i++) {
        KeepRule k;
        BFC_TRY(rule_of(g, reps[i], w.col_l, w.col_r, k, s));
        BFC_TRY(keep_and_scan(g, k, w, false, s));
        unsigned long long *o = st + 5 * (uint64_t)i;
        if (g->n_left) k_kept_stats<<<gl, 256, 0, s>>>(g->off_l, g->n_left, w.fl, o);
        if (g->n_right) k_kept_stats<<<gr, 256, 0, s>>>(g->off_r, g->n_right, w.fr, o + 2);
        k_kept_total<<<1, 64, 0, s>>>(w.fl, g->n_edges, o + 4);
        BFC_HIP(hipGetLastError());
    }
    std::vector<unsigned long long> h(5 * (size_t)nrep);
    BFC_HIP(hipMemcpyAsync(h.data(), st, h.size() * 8, hipMemcpyDeviceToHost, s));
    BFC_HIP(hipStreamSynchronize(s));
    for (uint32_t i = 0; i < nrep; i++) {
        const unsigned long long *o = &h[5 * (size_t)i];
        h_info[i].kept = o[4];
        h_info[i].n_left = (uint32_t)o[0];
        h_info[i].sumsq_left = o[1];
        h_info[i].n_right = (uint32_t)o[2];
        h_info[i].sumsq_right = o[3];
    }
    return BFC_OK;
}

int bfc_spar_batch_ws_size(const bfc_graph *g, uint32_t nrep, const bfc_replica *reps,
                           const bfc_replica_info *h_info, size_t *bytes) {
    if (!g || !h_info || !bytes) return BFC_E_NULL;
    BFC_TRY(check_replicas(nrep, reps));
    Carver c(nullptr, 0);
    BatchWs w;
    UnionLayout u;
    BFC_TRY(carve_batch(c, g, nrep, h_info, w, u));
    *bytes = c.used;
    return BFC_OK;
}

int bfc_spar_batch(const bfc_graph *g, uint32_t nrep, const bfc_replica *reps,
                   const bfc_replica_info *h_info, const bfc_tuning *tuning, uint64_t *d_beta,
                   double *d_est, void *d_ws, size_t ws_bytes, hipStream_t s) {
    if (!g || !h_info || !d_beta || !d_est || !d_ws) return BFC_E_NULL;
    BFC_TRY(check_replicas(nrep, reps));
    if (!aligned256(d_ws) || ((uintptr_t)d_beta & 7) || ((uintptr_t)d_est & 7)) return BFC_E_ALIGN;
    Carver c(d_ws, ws_bytes);
    BatchWs w;
    UnionLayout u;
    BFC_TRY(carve_batch(c, g, nrep, h_info, w, u));
    if (!c.fits()) return BFC_E_WS_SMALL;
    k_zero_u32x<<<1, 64, 0, s>>>(w.bad, 1);
    BFC_TRY(keep_rows(g, w.k, s));
    const uint64_t m = g->n_edges;
    const uint32_t nl = g->n_left, nr = g->n_right;
    for (uint32_t i = 0; i < nrep; i++) {
        const bfc_replica &rep = reps[i];
        KeepRule k;
        BFC_TRY(rule_of(g, rep, w.k.col_l, w.k.col_r, k, s));
        BFC_TRY(keep_and_scan(g, k, w.k, true, s));
        k_check_part<<<1, 64, 0, s>>>(w.k.fl, m, w.k.ml, nl, w.k.mr, nr, h_info[i].kept,
                                      h_info[i].n_left, h_info[i].n_right, w.bad);
        if (m) {
            // part i: its start side's rows into the union L (with cross
            // positions), the other side's into the union R
            const bool sw = u.swapped[i];
            EmitArgs el = {g->off_l, g->adj_l, g->xpos_l, w.k.fl, w.k.fr, w.k.ml, w.k.mr, nl,
                           u.ebase[i], sw ? u.vr[i] : u.vl[i], sw ? u.vl[i] : u.vr[i],
                           sw ? w.off_r : w.off_l, sw ? w.adj_r : w.adj_l,
                           sw ? nullptr : w.xpos_l, w.bad};
            EmitArgs er = {g->off_r, g->adj_r, g->xpos_r, w.k.fr, w.k.fl, w.k.mr, w.k.ml, nr,
                           u.ebase[i], sw ? u.vl[i] : u.vr[i], sw ? u.vr[i] : u.vl[i],
                           sw ? w.off_l : w.off_r, sw ? w.adj_l : w.adj_r,
                           sw ? w.xpos_l : nullptr, w.bad};
            BFC_TRY(emit(el, m, s));
            BFC_TRY(emit(er, m, s));
        }
        double div = 0.0, mul = 0.0;
        if (rep.kind == BFC_REPLICA_ESPAR) {
            div = (rep.p * rep.p) * (rep.p * rep.p);
        } else {
            const double N = (double)rep.ncolors;
            mul = N * N * N;
        }
        k_part_meta<<<1, 64, 0, s>>>(i, u.vl[i], div, mul, w.part_l, w.div, w.mul);
        BFC_HIP(hipGetLastError());
    }
    k_union_finish<<<grid_for((u.NL > u.NR ? u.NL : u.NR) + 1), 256, 0, s>>>(
        w.off_l, (uint32_t)u.NL, w.off_r, (uint32_t)u.NR, (uint32_t)u.M, w.part_l, nrep, w.bad);
    BFC_HIP(hipGetLastError());
    bfc_graph h = union_graph(g, u, w.off_l, w.adj_l, w.xpos_l, w.off_r, w.adj_r);
    BFC_TRY(bfc_exact_parts(&h, nrep, w.part_l, tuning, d_beta, w.work, w.work_bytes, s));
    k_est_batch<<<grid_for(nrep), 256, 0, s>>>((unsigned long long *)d_beta, w.div, w.mul, nrep,
                                               w.bad, d_est);
    BFC_HIP(hipGetLastError());
    return BFC_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ host: samplers
namespace bfc {

struct SampWs {
    ProbFlags *flags;
    unsigned long long *w, *pre, *scan_tmp, *draw, *cnt_l, *cnt_r, *cnt_e;
    uint32_t *wdraw, *pos;
    uint8_t *mark_l, *mark_r;
    double *parts;
    void *local;
    size_t local_bytes;
};

static int carve_samp(Carver &c, const bfc_graph *g, uint64_t n, uint64_t k, int edges,
                      SampWs &w) {
    size_t lb = 0, t;
    BFC_TRY(local_ws_size(g, BFC_SIDE_L, &t));
    lb = t;
    BFC_TRY(local_ws_size(g, BFC_SIDE_R, &t));
    lb = t > lb ? t : lb;
    w.flags = c.take<ProbFlags>(1);
    w.w = c.take<unsigned long long>(pad64(n));
    w.pre = c.take<unsigned long long>(pad64(n));
    w.scan_tmp = c.take<unsigned long long>((n + S64_TILE - 1) / S64_TILE + 64);
    w.draw = c.take<unsigned long long>(pad64(k));
    w.wdraw = c.take<uint32_t>(pad64(k));
    w.parts = c.take<double>((k + COMBINE_BLOCK - 1) / COMBINE_BLOCK + 1024);
    w.mark_l = c.take<uint8_t>(pad64(g->n_left));
    w.mark_r = c.take<uint8_t>(pad64(g->n_right));
    if (edges) {
        w.cnt_e = c.take<unsigned long long>(pad64(g->n_edges));
        w.pos = c.take<uint32_t>(pad64(g->n_edges));
        w.cnt_l = w.cnt_r = nullptr;
    } else {
        w.cnt_l = c.take<unsigned long long>(pad64(g->n_left));
        w.cnt_r = c.take<unsigned long long>(pad64(g->n_right));
        w.cnt_e = nullptr;
        w.pos = nullptr;
    }
    w.local_bytes = lb;
    w.local = c.take<char>(lb);
    return BFC_OK;
}

// The draw buffers of carve_samp alone (bfc_vsamp_draws).
static void carve_draws(Carver &c, uint64_t n, uint64_t k, SampWs &w) {
    w = SampWs{};
    w.flags = c.take<ProbFlags>(1);
    w.w = c.take<unsigned long long>(pad64(n));
    w.pre = c.take<unsigned long long>(pad64(n));
    w.scan_tmp = c.take<unsigned long long>((n + S64_TILE - 1) / S64_TILE + 64);
    w.draw = c.take<unsigned long long>(pad64(k));
    w.wdraw = c.take<uint32_t>(pad64(k));
}

// Fast-eBFC sampler: the draw buffers of carve_samp, the edge position map
// and the per-draw endpoints.
static void carve_fast(Carver &c, uint64_t m, uint64_t k, SampWs &w, uint32_t *&ea,
                       uint32_t *&ex, double *&terms) {
    w = SampWs{};
    w.flags = c.take<ProbFlags>(1);
    w.w = c.take<unsigned long long>(pad64(m));
    w.pre = c.take<unsigned long long>(pad64(m));
    w.scan_tmp = c.take<unsigned long long>((m + S64_TILE - 1) / S64_TILE + 64);
    w.draw = c.take<unsigned long long>(pad64(k));
    w.wdraw = c.take<uint32_t>(pad64(k));
    w.parts = c.take<double>((k + COMBINE_BLOCK - 1) / COMBINE_BLOCK + 1024);
    w.pos = c.take<uint32_t>(pad64(m));
    ea = c.take<uint32_t>(pad64(k));
    ex = c.take<uint32_t>(pad64(k));
    terms = c.take<double>(pad64(k));
}

// WSamp: prefix sums of C(d,2) over the n vertices, scan scratch, partial sums.
static void carve_wsamp(Carver &c, uint64_t n, unsigned long long *&pre,
                        unsigned long long *&tmp, unsigned long long *&parts) {
    pre = c.take<unsigned long long>(pad64(n));
    tmp = c.take<unsigned long long>((n + S64_TILE - 1) / S64_TILE + 64);
    parts = c.take<unsigned long long>(256);
}

// Weights, prefix sums and k draws over n items.  Asynchronous: invalid
// probabilities are detected on the device (the estimate becomes NaN);
// bfc_probs_check reports them to the host.
static int sample_draws(const double *d_probs, uint64_t n, uint64_t k, uint64_t seed,
                        uint32_t tag, SampWs &w, hipStream_t s) {
    k_zero_flags<<<1, 64, 0, s>>>(w.flags);
    if (d_probs) {
        k_prob_scan<<<grid_for(n), 256, 0, s>>>(d_probs, n, w.flags);
        k_quantise<<<grid_for(n), 256, 0, s>>>(d_probs, n, w.flags, w.w, w.pre);
        BFC_HIP(hipGetLastError());
        BFC_TRY(scan_u64_inclusive(w.pre, n, w.scan_tmp, s));
    }
    k_draw<<<grid_for(k), 256, 0, s>>>(k, n, seed, tag, d_probs ? w.pre : nullptr, w.w, w.draw,
                                       w.wdraw);
    BFC_HIP(hipGetLastError());
    return BFC_OK;
}

static int finish_estimate(uint64_t k, uint64_t n, const unsigned long long *counts, bool weighted,
                           SampWs &w, double *d_est, hipStream_t s) {
    k_combine<<<1, 256, 0, s>>>(k, n, counts, w.wdraw, weighted ? w.pre : nullptr, w.parts,
                                w.flags, d_est);
    BFC_HIP(hipGetLastError());
    return BFC_OK;
}

}  // namespace bfc

extern "C" {

int bfc_probs_check_ws_size(size_t *bytes) {
    if (!bytes) return BFC_E_NULL;
    *bytes = 256;
    return BFC_OK;
}

int bfc_probs_check(const double *d_probs, uint64_t n, void *d_ws, size_t ws_bytes,
                    hipStream_t s) {
    if (!d_probs || !d_ws) return BFC_E_NULL;
    if (n == 0) return BFC_E_ARG;
    if (!aligned256(d_ws)) return BFC_E_ALIGN;
    if (ws_bytes < sizeof(ProbFlags)) return BFC_E_WS_SMALL;
    ProbFlags *f = (ProbFlags *)d_ws;
    k_zero_flags<<<1, 64, 0, s>>>(f);
    k_prob_scan<<<grid_for(n), 256, 0, s>>>(d_probs, n, f);
    BFC_HIP(hipGetLastError());
    ProbFlags hf;
    BFC_HIP(hipMemcpyAsync(&hf, f, sizeof(hf), hipMemcpyDeviceToHost, s));
    BFC_HIP(hipStreamSynchronize(s));
    return (hf.bad || hf.max_bits == 0) ? BFC_E_PROBS : BFC_OK;
}

int bfc_vsamp_ws_size(const bfc_graph *g, uint64_t k, size_t *bytes) {
    if (!g || !bytes) return BFC_E_NULL;
    Carver c(nullptr, 0);
    SampWs w;
    BFC_TRY(carve_samp(c, g, (uint64_t)g->n_left + g->n_right, k, 0, w));
    *bytes = c.used;
    return BFC_OK;
}

int bfc_vsamp(const bfc_graph *g, const double *d_probs, uint64_t k, uint64_t seed,
              uint32_t *d_ids, uint64_t *d_counts, double *d_est, void *d_ws, size_t ws_bytes,
              hipStream_t s) {
    if (!g || !d_ids || !d_counts || !d_est || !d_ws) return BFC_E_NULL;
    const uint64_t n = (uint64_t)g->n_left + g->n_right;
    if (k == 0 || n == 0) return BFC_E_ARG;
    if (!aligned256(d_ws) || ((uintptr_t)d_counts & 7) || ((uintptr_t)d_est & 7)) return BFC_E_ALIGN;
    Carver c(d_ws, ws_bytes);
    SampWs w;
    BFC_TRY(carve_samp(c, g, n, k, 0, w));
    if (!c.fits()) return BFC_E_WS_SMALL;
    BFC_TRY(sample_draws(d_probs, n, k, seed, TAG_VDRAW, w, s));
    k_zero_u32x<<<grid_for(pad64(g->n_left) / 4), 256, 0, s>>>((uint32_t *)w.mark_l,
                                                               pad64(g->n_left) / 4);
    k_zero_u32x<<<grid_for(pad64(g->n_right) / 4), 256, 0, s>>>((uint32_t *)w.mark_r,
                                                                pad64(g->n_right) / 4);
    k_mark_vertices<<<grid_for(k), 256, 0, s>>>(k, w.draw, g->n_left, g->rank_l, g->rank_r,
                                                w.mark_l, w.mark_r, d_ids);
    k_zero_u64x<<<grid_for(g->n_left), 256, 0, s>>>(w.cnt_l, g->n_left);
    k_zero_u64x<<<grid_for(g->n_right), 256, 0, s>>>(w.cnt_r, g->n_right);
    BFC_HIP(hipGetLastError());
    // vBFC of every drawn vertex: the local walk from each side over the
    // marked starts only, per-vertex counts only
    if (g->n_left)
        BFC_TRY(local_run(g, BFC_SIDE_L, w.mark_l, (uint64_t *)w.cnt_l, nullptr, nullptr, w.local,
                          w.local_bytes, s));
    if (g->n_right)
        BFC_TRY(local_run(g, BFC_SIDE_R, w.mark_r, nullptr, (uint64_t *)w.cnt_r, nullptr, w.local,
                          w.local_bytes, s));
    k_gather_vertex<<<grid_for(k), 256, 0, s>>>(k, d_ids, g->n_left, w.cnt_l, w.cnt_r,
                                                (unsigned long long *)d_counts);
    BFC_HIP(hipGetLastError());
    return finish_estimate(k, n, (unsigned long long *)d_counts, d_probs != nullptr, w, d_est, s);
}

int bfc_vsamp_draws_ws_size(const bfc_graph *g, uint64_t k, size_t *bytes) {
    if (!g || !bytes) return BFC_E_NULL;
    const uint64_t n = (uint64_t)g->n_left + g->n_right;
    Carver c(nullptr, 0);
    SampWs w;
    carve_draws(c, n, k, w);
    *bytes = c.used;
    return BFC_OK;
}

int bfc_vsamp_draws(const bfc_graph *g, const double *d_probs, uint64_t k, uint64_t seed,
                    uint32_t *d_ids, uint32_t *d_weights, uint64_t *d_total_weight, void *d_ws,
                    size_t ws_bytes, hipStream_t s) {
    if (!g || !d_ids || !d_ws) return BFC_E_NULL;
    const uint64_t n = (uint64_t)g->n_left + g->n_right;
    if (k == 0 || n == 0) return BFC_E_ARG;
    if (!aligned256(d_ws) || ((uintptr_t)d_total_weight & 7)) return BFC_E_ALIGN;
    Carver c(d_ws, ws_bytes);
    SampWs w;
    carve_draws(c, n, k, w);
    if (!c.fits()) return BFC_E_WS_SMALL;
    BFC_TRY(sample_draws(d_probs, n, k, seed, TAG_VDRAW, w, s));
    k_draw_ids<<<grid_for(k), 256, 0, s>>>(k, n, w.draw, w.wdraw, d_probs ? w.pre : nullptr,
                                           d_ids, d_weights,
                                           (unsigned long long *)d_total_weight);
    BFC_HIP(hipGetLastError());
    return BFC_OK;
}

int bfc_esamp_ws_size(const bfc_graph *g, uint64_t k, size_t *bytes) {
    if (!g || !bytes) return BFC_E_NULL;
    Carver c(nullptr, 0);
    SampWs w;
    BFC_TRY(carve_samp(c, g, g->n_edges, k, 1, w));
    *bytes = c.used;
    return BFC_OK;
}

int bfc_esamp(const bfc_graph *g, const double *d_probs, uint64_t k, uint64_t seed,
              uint64_t *d_eids, uint64_t *d_counts, double *d_est, void *d_ws, size_t ws_bytes,
              hipStream_t s) {
    if (!g || !d_eids || !d_counts || !d_est || !d_ws) return BFC_E_NULL;
    const uint64_t m = g->n_edges;
    if (k == 0 || m == 0) return BFC_E_ARG;
    if (!aligned256(d_ws) || ((uintptr_t)d_counts & 7) || ((uintptr_t)d_eids & 7) ||
        ((uintptr_t)d_est & 7))
        return BFC_E_ALIGN;
    Carver c(d_ws, ws_bytes);
    SampWs w;
    BFC_TRY(carve_samp(c, g, m, k, 1, w));
    if (!c.fits()) return BFC_E_WS_SMALL;
    BFC_TRY(sample_draws(d_probs, m, k, seed, TAG_EDRAW, w, s));
    // eBFC of every drawn edge: walk from the side the paper's rule picks,
    // over the starts of the drawn edges, per-edge counts
    const int side = bfc_side_used(g, BFC_SIDE_AUTO);
    const bool from_r = side == BFC_SIDE_R;
    const uint32_t nA = from_r ? g->n_right : g->n_left;
    uint8_t *mark = from_r ? w.mark_r : w.mark_l;
    k_zero_u32x<<<grid_for(pad64(nA) / 4), 256, 0, s>>>((uint32_t *)mark, pad64(nA) / 4);
    k_pos_of_edge<<<grid_for(m), 256, 0, s>>>(from_r ? g->eid_r : g->eid_l, m, w.pos);
    k_mark_edges<<<grid_for(k), 256, 0, s>>>(k, w.draw, w.pos, from_r ? g->off_r : g->off_l, nA,
                                             mark);
    k_zero_u64x<<<grid_for(m), 256, 0, s>>>(w.cnt_e, m);
    BFC_HIP(hipGetLastError());
    BFC_TRY(local_run(g, side, mark, nullptr, nullptr, (uint64_t *)w.cnt_e, w.local, w.local_bytes,
                      s));
    k_gather_edge<<<grid_for(k), 256, 0, s>>>(k, w.draw, w.cnt_e, (unsigned long long *)d_counts,
                                              (unsigned long long *)d_eids);
    BFC_HIP(hipGetLastError());
    return finish_estimate(k, m, (unsigned long long *)d_counts, d_probs != nullptr, w, d_est, s);
}

int bfc_esamp_fast_ws_size(const bfc_graph *g, uint64_t k, size_t *bytes) {
    if (!g || !bytes) return BFC_E_NULL;
    Carver c(nullptr, 0);
    SampWs w;
    uint32_t *ea, *ex;
    double *terms;
    carve_fast(c, g->n_edges, k, w, ea, ex, terms);
    *bytes = c.used;
    return BFC_OK;
}

int bfc_esamp_fast(const bfc_graph *g, const double *d_probs, uint64_t k, uint32_t alpha,
                   uint64_t seed, uint64_t *d_eids, uint32_t *d_hits, double *d_est, void *d_ws,
                   size_t ws_bytes, hipStream_t s) {
    if (!g || !d_eids || !d_hits || !d_est || !d_ws) return BFC_E_NULL;
    const uint64_t m = g->n_edges;
    if (k == 0 || k > 0xFFFFFFFFull || alpha == 0 || m == 0) return BFC_E_ARG;
    if (!aligned256(d_ws) || ((uintptr_t)d_eids & 7) || ((uintptr_t)d_hits & 3) ||
        ((uintptr_t)d_est & 7))
        return BFC_E_ALIGN;
    Carver c(d_ws, ws_bytes);
    SampWs w;
    uint32_t *ea, *ex;
    double *terms;
    carve_fast(c, m, k, w, ea, ex, terms);
    if (!c.fits()) return BFC_E_WS_SMALL;
    BFC_TRY(sample_draws(d_probs, m, k, seed, TAG_EDRAW, w, s));
    k_pos_of_edge<<<grid_for(m), 256, 0, s>>>(g->eid_l, m, w.pos);
    k_fast_setup<<<grid_for(k), 256, 0, s>>>(k, w.draw, w.pos, g->off_l, g->n_left, g->adj_l, ea,
                                             ex, d_hits, (unsigned long long *)d_eids);
    FastArgs f = {g->off_l, g->adj_l, g->off_r, g->adj_r, ea, ex, k, seed, alpha};
    const uint64_t units = k * ((alpha + WAVE - 1) / WAVE);
    const uint64_t blocks = (units + 3) / 4;
    k_fast_trials<<<(unsigned)(blocks < 16384 ? blocks : 16384), 256, 0, s>>>(f, d_hits);
    k_fast_terms<<<grid_for(k), 256, 0, s>>>(f, m, d_hits, w.wdraw, d_probs ? w.pre : nullptr,
                                             terms);
    k_block_sums<<<grid_for((k + COMBINE_BLOCK - 1) / COMBINE_BLOCK, 64), 64, 0, s>>>(terms, k,
                                                                                  w.parts);
    k_fast_total<<<1, 64, 0, s>>>(k, alpha, w.parts, d_probs ? w.flags : nullptr, d_est);
    BFC_HIP(hipGetLastError());
    return BFC_OK;
}

int bfc_wsamp_ws_size(const bfc_graph *g, uint64_t k, size_t *bytes) {
    if (!g || !bytes) return BFC_E_NULL;
    Carver c(nullptr, 0);
    unsigned long long *pre, *tmp, *parts;
    carve_wsamp(c, (uint64_t)g->n_left + g->n_right, pre, tmp, parts);
    (void)k;
    *bytes = c.used;
    return BFC_OK;
}

int bfc_wsamp(const bfc_graph *g, uint64_t k, uint64_t seed, uint32_t *d_mids, uint32_t *d_ends,
              uint64_t *d_counts, double *d_est, void *d_ws, size_t ws_bytes, hipStream_t s) {
    if (!g || !d_mids || !d_ends || !d_counts || !d_est || !d_ws) return BFC_E_NULL;
    const uint64_t n = (uint64_t)g->n_left + g->n_right;
    const uint64_t W = g->wedges_mid_l + g->wedges_mid_r;
    if (k == 0 || k > 0xFFFFFFFFull || W == 0) return BFC_E_ARG;
    if (!aligned256(d_ws) || ((uintptr_t)d_counts & 7) || ((uintptr_t)d_est & 7) ||
        ((uintptr_t)d_mids & 3) || ((uintptr_t)d_ends & 3))
        return BFC_E_ALIGN;
    Carver c(d_ws, ws_bytes);
    unsigned long long *pre, *tmp, *parts;
    carve_wsamp(c, n, pre, tmp, parts);
    if (!c.fits()) return BFC_E_WS_SMALL;
    k_wedge_weights<<<grid_for(n), 256, 0, s>>>(g->n_left, g->n_right, g->rank_l, g->rank_r,
                                                g->off_l, g->off_r, pre);
    BFC_HIP(hipGetLastError());
    BFC_TRY(scan_u64_inclusive(pre, n, tmp, s));
    WsampArgs a = {g->off_l, g->adj_l, g->off_r, g->adj_r, g->rank_l, g->rank_r, g->id_l,
                   g->id_r, pre, n, W, k, seed, g->n_left};
    const uint64_t blocks = (k + 3) / 4;
    k_wsamp<<<(unsigned)(blocks < 16384 ? blocks : 16384), 256, 0, s>>>(
        a, d_mids, d_ends, (unsigned long long *)d_counts);
    k_zero_u64<<<1, 64, 0, s>>>(parts);
    const uint64_t sb = (k + 255) / 256;
    k_wsamp_sum<<<(unsigned)(sb < 2048 ? sb : 2048), 256, 0, s>>>(
        k, (const unsigned long long *)d_counts, parts);
    k_wsamp_est<<<1, 64, 0, s>>>(k, (double)W, parts, d_est);
    BFC_HIP(hipGetLastError());
    return BFC_OK;
}

int bfc_spar_threshold(int kind, double B, uint32_t max_deg, double *p, uint32_t *ncolors) {
    if (!p || !ncolors) return BFC_E_NULL;
    if (!(B == B)) return BFC_E_ARG;
    const double D = (double)max_deg;
    *p = 1.0;
    *ncolors = 1;
    if (kind == BFC_REPLICA_ESPAR) {
        if (B <= 0.0) return BFC_OK;
        double b = pow(24.0 / B, 0.25);
        b = fmax(b, sqrt(24.0 * D / B));
        b = fmax(b, 24.0 * D * D / B);
        *p = b < 1.0 ? b : 1.0;
        return BFC_OK;
    }
    if (kind == BFC_REPLICA_CLRSPAR) {
        if (B <= 0.0) return BFC_OK;
        double b = pow(32.0 / B, 1.0 / 3.0);
        b = fmax(b, sqrt(32.0 * D / B));
        b = fmax(b, 32.0 * D * D / B);
        if (b >= 1.0) return BFC_OK;
        double f = floor(1.0 / b);            // then the largest N with 1/N > b
        uint64_t n = f > 4294967295.0 ? 4294967295ull : (uint64_t)f;
        if (n < 1) n = 1;
        while (n > 1 && !(1.0 / (double)n > b)) n--;
        while (n < 4294967295ull && 1.0 / (double)(n + 1) > b) n++;
        *ncolors = (uint32_t)n;
        *p = 1.0 / (double)n;
        return BFC_OK;
    }
    return BFC_E_ARG;
}

int bfc_eps_delta_plan(double eps, double delta, uint32_t *groups, uint32_t *per_group) {
    if (!groups || !per_group) return BFC_E_NULL;
    if (!(eps > 0.0 && eps <= 1.0) || !(delta > 0.0 && delta < 1.0)) return BFC_E_ARG;
    const double r = ceil(3.0 / (2.0 * eps * eps));
    double g = ceil(8.0 * log(1.0 / delta));
    if (fmod(g, 2.0) == 0.0) g += 1.0;
    if (r > 4294967295.0 || g > (double)MOM_MAX_GROUPS) return BFC_E_ARG;
    *groups = (uint32_t)g;
    *per_group = (uint32_t)r;
    return BFC_OK;
}

int bfc_median_of_means(const double *d_x, uint32_t groups, uint32_t per_group, double *d_means,
                        double *d_median, hipStream_t s) {
    if (!d_x || !d_means || !d_median) return BFC_E_NULL;
    if (groups == 0 || per_group == 0 || groups > MOM_MAX_GROUPS) return BFC_E_ARG;
    if (((uintptr_t)d_x & 7) || ((uintptr_t)d_means & 7) || ((uintptr_t)d_median & 7))
        return BFC_E_ALIGN;
    k_median_of_means<<<1, 256, 0, s>>>(d_x, groups, per_group, d_means, d_median);
    BFC_HIP(hipGetLastError());
    return BFC_OK;
}

}  // extern "C"
