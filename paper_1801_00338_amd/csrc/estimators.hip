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
// Every L row, one wave per row: the keep flag of each edge (l, r) by ids.
struct FilterArgs {
    const uint32_t *off_l, *adj_l, *id_l, *id_r;
    uint32_t nl;
    int kind;                   // 0 = ESpar, 1 = ClrSpar
    uint64_t seed, thresh;      // ESpar: keep iff x < thresh (keep_all overrides)
    int keep_all;
    const uint32_t *col_l, *col_r;  // ClrSpar colours by id
};

__device__ inline uint32_t keep_edge(const FilterArgs &f, uint32_t l, uint32_t r) {
    if (f.keep_all) return 1u;
    if (f.kind == 0) {
        uint32_t o[4];
        philox(l, r, TAG_ESPAR, 0, f.seed, o);
        const uint64_t x = (uint64_t)o[0] | ((uint64_t)o[1] << 32);
        return x < f.thresh;
    }
    return f.col_l[l] == f.col_r[r];
}

__global__ __launch_bounds__(256) void k_filter(FilterArgs f, uint32_t *flag) {
    const uint32_t lane = threadIdx.x & (WAVE - 1), wpb = blockDim.x / WAVE;
    for (uint32_t u = blockIdx.x * wpb + threadIdx.x / WAVE; u < f.nl; u += gridDim.x * wpb) {
        const uint32_t l = f.id_l[u];
        for (uint32_t k = f.off_l[u] + lane; k < f.off_l[u + 1]; k += WAVE)
            flag[k] = keep_edge(f, l, f.id_r[f.adj_l[k]]);
    }
}

// Kept edges, compacted by the inclusive scan of the flags (same row walk);
// at most `cap` of them are written.
__global__ __launch_bounds__(256) void k_compact(FilterArgs f, const uint32_t *scan1,
                                                 uint32_t *kl, uint32_t *kr, uint32_t cap) {
    const uint32_t lane = threadIdx.x & (WAVE - 1), wpb = blockDim.x / WAVE;
    for (uint32_t u = blockIdx.x * wpb + threadIdx.x / WAVE; u < f.nl; u += gridDim.x * wpb) {
        const uint32_t l = f.id_l[u];
        for (uint32_t k = f.off_l[u] + lane; k < f.off_l[u + 1]; k += WAVE) {
            const uint32_t prev = k ? scan1[k - 1] : 0;
            if (scan1[k] != prev && prev < cap) {
                kl[prev] = l;
                kr[prev] = f.id_r[f.adj_l[k]];
            }
        }
    }
}

__global__ void k_colours(uint32_t n, uint32_t side, uint32_t N, uint64_t seed, uint32_t *col) {
    for (uint64_t v = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; v < n;
         v += (uint64_t)gridDim.x * blockDim.x)
        col[v] = colour_of(seed, side, v, N);
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

__global__ void k_quantise(const double *probs, uint64_t n, const ProbFlags *f,
                           unsigned long long *w) {
    const double mx = __longlong_as_double((long long)f->max_bits);
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const double p = probs[i];
        unsigned long long q = 0;
        if (p > 0.0) {
            const double s = floor(p / mx * 4294967295.0);
            const uint32_t v = (uint32_t)s;
            q = v < 1 ? 1 : v;
        }
        w[i] = q;
    }
}

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
            *est = ((double)t * (double)n) / (4.0 * (double)k);
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

__global__ void k_fast_total(uint64_t k, uint32_t alpha, const double *parts, double *est) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const uint64_t nb = (k + COMBINE_BLOCK - 1) / COMBINE_BLOCK;
        double total = 0.0;
        for (uint64_t b = 0; b < nb; b++) total += parts[b];
        *est = total / ((double)k * (double)alpha);
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
struct SparWs {
    uint32_t *flag, *scan_tmp, *kl, *kr, *col_l, *col_r;
    void *storage;
    size_t storage_bytes;
    void *work;                 // graph build workspace, then the exact count's
    size_t work_bytes;
};

static int carve_spar(Carver &c, uint32_t nl, uint32_t nr, uint64_t m, SparWs &w) {
    size_t sb, bb;
    BFC_TRY(bfc_graph_storage_size(nl, nr, m, &sb));
    BFC_TRY(bfc_graph_build_ws_size(nl, nr, m, &bb));
    const size_t eb = exact_ws_bound(nl, nr, m);
    w.flag = c.take<uint32_t>(pad64(m));
    w.scan_tmp = c.take<uint32_t>(scan_tmp_elems(m));
    w.kl = c.take<uint32_t>(pad64(m));
    w.kr = c.take<uint32_t>(pad64(m));
    w.col_l = c.take<uint32_t>(pad64(nl));
    w.col_r = c.take<uint32_t>(pad64(nr));
    w.storage_bytes = sb;
    w.storage = c.take<char>(sb);
    w.work_bytes = bb > eb ? bb : eb;
    w.work = c.take<char>(w.work_bytes);
    return BFC_OK;
}

// Filter, compact, rebuild and count the kept graph.
static int sparsify_count(const bfc_graph *g, FilterArgs f, SparWs &w, uint64_t *d_beta,
                          uint64_t *kept, hipStream_t s) {
    const uint64_t m = g->n_edges;
    uint64_t mk = 0;
    if (m) {
        unsigned gr = grid_for(g->n_left, 4);
        if (gr > 8192) gr = 8192;
        k_filter<<<gr, 256, 0, s>>>(f, w.flag);
        BFC_HIP(hipGetLastError());
        BFC_TRY(scan_u32_inclusive(w.flag, w.flag, m, w.scan_tmp, s));
        k_compact<<<gr, 256, 0, s>>>(f, w.flag, w.kl, w.kr, 0xFFFFFFFFu);
        BFC_HIP(hipGetLastError());
        uint32_t last = 0;
        BFC_HIP(hipMemcpyAsync(&last, w.flag + (m - 1), 4, hipMemcpyDeviceToHost, s));
        BFC_HIP(hipStreamSynchronize(s));
        mk = last;
    }
    if (kept) *kept = mk;
    bfc_graph h;
    BFC_TRY(bfc_graph_build(g->n_left, g->n_right, mk, w.kl, w.kr, w.storage, w.storage_bytes,
                            w.work, w.work_bytes, s, &h));
    return bfc_exact(&h, BFC_SIDE_AUTO, d_beta, w.work, w.work_bytes, s);
}

}  // namespace bfc

using namespace bfc;

extern "C" {

int bfc_spar_ws_size(const bfc_graph *g, size_t *bytes) {
    if (!g || !bytes) return BFC_E_NULL;
    Carver c(nullptr, 0);
    SparWs w;
    BFC_TRY(carve_spar(c, g->n_left, g->n_right, g->n_edges, w));
    *bytes = c.used;
    return BFC_OK;
}

int bfc_espar(const bfc_graph *g, double p, uint64_t seed, uint64_t *d_beta, double *d_est,
              uint64_t *kept_edges, void *d_ws, size_t ws_bytes, hipStream_t s) {
    if (!g || !d_beta || !d_est || !d_ws) return BFC_E_NULL;
    if (!(p > 0.0) || !(p <= 1.0)) return BFC_E_ARG;
    if (!aligned256(d_ws) || ((uintptr_t)d_beta & 7) || ((uintptr_t)d_est & 7)) return BFC_E_ALIGN;
    Carver c(d_ws, ws_bytes);
    SparWs w;
    BFC_TRY(carve_spar(c, g->n_left, g->n_right, g->n_edges, w));
    if (!c.fits()) return BFC_E_WS_SMALL;
    FilterArgs f = {};
    f.off_l = g->off_l; f.adj_l = g->adj_l; f.id_l = g->id_l; f.id_r = g->id_r;
    f.nl = g->n_left;
    f.kind = 0;
    f.seed = seed;
    f.keep_all = p >= 1.0;
    f.thresh = f.keep_all ? 0 : (uint64_t)ldexp(p, 64);
    BFC_TRY(sparsify_count(g, f, w, d_beta, kept_edges, s));
    k_est_scale<<<1, 64, 0, s>>>((unsigned long long *)d_beta, (p * p) * (p * p), 0.0, d_est);
    BFC_HIP(hipGetLastError());
    return BFC_OK;
}

int bfc_clrspar(const bfc_graph *g, uint32_t ncolors, uint64_t seed, uint64_t *d_beta,
                double *d_est, uint64_t *kept_edges, void *d_ws, size_t ws_bytes, hipStream_t s) {
    if (!g || !d_beta || !d_est || !d_ws) return BFC_E_NULL;
    if (ncolors == 0) return BFC_E_ARG;
    if (!aligned256(d_ws) || ((uintptr_t)d_beta & 7) || ((uintptr_t)d_est & 7)) return BFC_E_ALIGN;
    Carver c(d_ws, ws_bytes);
    SparWs w;
    BFC_TRY(carve_spar(c, g->n_left, g->n_right, g->n_edges, w));
    if (!c.fits()) return BFC_E_WS_SMALL;
    FilterArgs f = {};
    f.off_l = g->off_l; f.adj_l = g->adj_l; f.id_l = g->id_l; f.id_r = g->id_r;
    f.nl = g->n_left;
    f.kind = 1;
    f.seed = seed;
    f.keep_all = ncolors == 1;
    f.col_l = w.col_l;
    f.col_r = w.col_r;
    if (!f.keep_all) {
        if (g->n_left) k_colours<<<grid_for(g->n_left), 256, 0, s>>>(g->n_left, 0, ncolors, seed, w.col_l);
        if (g->n_right) k_colours<<<grid_for(g->n_right), 256, 0, s>>>(g->n_right, 1, ncolors, seed, w.col_r);
        BFC_HIP(hipGetLastError());
    }
    BFC_TRY(sparsify_count(g, f, w, d_beta, kept_edges, s));
    const double N = (double)ncolors;
    k_est_scale<<<1, 64, 0, s>>>((unsigned long long *)d_beta, 0.0, N * N * N, d_est);
    BFC_HIP(hipGetLastError());
    return BFC_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ host: replica batches
// Many ESpar / ClrSpar replicas of one graph counted in one launch: each
// replica's kept edges are compacted into a shared pool with its vertices
// renumbered densely (isolated vertices dropped: they carry no butterfly),
// the replicas become the parts of one disjoint union (each oriented by
// ExactBFC's side rule) and bfc_exact_parts counts them together.  Every
// replica's count and estimate equal those of bfc_espar / bfc_clrspar with
// the same parameters and seed.
namespace bfc {

__global__ void k_mark_ends(const uint32_t *kl, const uint32_t *kr, uint64_t mk, uint32_t *ml,
                            uint32_t *mr) {
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < mk;
         e += (uint64_t)gridDim.x * blockDim.x) {
        ml[kl[e]] = 1u;
        mr[kr[e]] = 1u;
    }
}

// New id = (inclusive scan of the marks at the old id) - 1.
__global__ void k_renumber(uint32_t *kl, uint32_t *kr, uint64_t mk, const uint32_t *sl,
                           const uint32_t *sr) {
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < mk;
         e += (uint64_t)gridDim.x * blockDim.x) {
        kl[e] = sl[kl[e]] - 1u;
        kr[e] = sr[kr[e]] - 1u;
    }
}

__global__ void k_store_last(const uint32_t *scan, uint64_t n, uint32_t *out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *out = n ? scan[n - 1] : 0u;
}

__global__ void k_zero32(uint32_t *p, uint64_t n) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

__global__ void k_est_batch(const unsigned long long *beta, const double *div, const double *mul,
                            uint32_t n, double *est) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const double b = (double)beta[i];
        est[i] = div[i] != 0.0 ? b / div[i] : b * mul[i];
    }
}

// Degrees of the kept edges (flags from k_filter), by ids.
__global__ __launch_bounds__(256) void k_kept_degrees(FilterArgs f, const uint32_t *flag,
                                                      uint32_t *deg_l, uint32_t *deg_r) {
    const uint32_t lane = threadIdx.x & (WAVE - 1), wpb = blockDim.x / WAVE;
    for (uint32_t u = blockIdx.x * wpb + threadIdx.x / WAVE; u < f.nl; u += gridDim.x * wpb) {
        const uint32_t l = f.id_l[u];
        for (uint32_t k = f.off_l[u] + lane; k < f.off_l[u + 1]; k += WAVE)
            if (flag[k]) {
                atomicAdd(&deg_l[l], 1u);
                atomicAdd(&deg_r[f.id_r[f.adj_l[k]]], 1u);
            }
    }
}

// out[0] += vertices of nonzero degree, out[1] += sum of squared degrees.
__global__ __launch_bounds__(256) void k_deg_stats(const uint32_t *deg, uint64_t n,
                                                   unsigned long long *out) {
    __shared__ unsigned long long red[256 / WAVE];
    unsigned long long c = 0, q = 0;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const unsigned long long d = deg[i];
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

__global__ void k_zero64(unsigned long long *p, uint64_t n) {
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

struct FilterWs {
    uint32_t *flag, *scan_tmp, *col_l, *col_r;
};

static void carve_filter(Carver &c, const bfc_graph *g, FilterWs &w) {
    w.flag = c.take<uint32_t>(pad64(g->n_edges));
    w.scan_tmp = c.take<uint32_t>(scan_tmp_elems(g->n_edges));
    w.col_l = c.take<uint32_t>(pad64(g->n_left));
    w.col_r = c.take<uint32_t>(pad64(g->n_right));
}

// Keep flags of replica `rep` in w.flag, then their inclusive scan.
static int filter_replica(const bfc_graph *g, const bfc_replica &rep, FilterWs &w,
                          FilterArgs &f, hipStream_t s) {
    f = FilterArgs{};
    f.off_l = g->off_l; f.adj_l = g->adj_l; f.id_l = g->id_l; f.id_r = g->id_r;
    f.nl = g->n_left;
    f.seed = rep.seed;
    if (rep.kind == BFC_REPLICA_ESPAR) {
        f.kind = 0;
        f.keep_all = rep.p >= 1.0;
        f.thresh = f.keep_all ? 0 : (uint64_t)ldexp(rep.p, 64);
    } else {
        f.kind = 1;
        f.keep_all = rep.ncolors == 1;
        f.col_l = w.col_l;
        f.col_r = w.col_r;
        if (!f.keep_all) {
            if (g->n_left)
                k_colours<<<grid_for(g->n_left), 256, 0, s>>>(g->n_left, 0, rep.ncolors, rep.seed,
                                                              w.col_l);
            if (g->n_right)
                k_colours<<<grid_for(g->n_right), 256, 0, s>>>(g->n_right, 1, rep.ncolors,
                                                               rep.seed, w.col_r);
        }
    }
    const uint64_t m = g->n_edges;
    if (m) {
        unsigned gr = grid_for(g->n_left, 4);
        if (gr > 8192) gr = 8192;
        k_filter<<<gr, 256, 0, s>>>(f, w.flag);
        BFC_HIP(hipGetLastError());
        BFC_TRY(scan_u32_inclusive(w.flag, w.flag, m, w.scan_tmp, s));
    }
    BFC_HIP(hipGetLastError());
    return BFC_OK;
}

struct BatchWs {
    FilterWs f;
    uint32_t *ml, *mr, *scan_tmp_v, *kl, *kr, *kept_dev, *sizes_dev, *part_l, *part_r;
    double *div, *mul;
    void *storage;
    size_t storage_bytes;
    void *work;
    size_t work_bytes;
};

// Sizes of the union: edges, vertices of each union side (each part enters
// with its start side as L: ExactBFC's rule on its own degrees), and the
// sums of the parts' vertex counts before orientation.
struct BatchSizes {
    uint64_t M, NL, NR, SL, SR;
};

static int batch_sizes(uint32_t nrep, const bfc_replica_info *info, BatchSizes &z) {
    z = BatchSizes{0, 0, 0, 0, 0};
    for (uint32_t i = 0; i < nrep; i++) {
        const bfc_replica_info &r = info[i];
        const bool sw = r.sumsq_left < r.sumsq_right;
        z.M += r.kept;
        z.NL += sw ? r.n_right : r.n_left;
        z.NR += sw ? r.n_left : r.n_right;
        z.SL += r.n_left;
        z.SR += r.n_right;
    }
    if (z.M > 0xFFFFFFFFull - ADJ_SLACK || z.NL > 0xFFFFFFFEull || z.NR > 0xFFFFFFFEull)
        return BFC_E_TOO_LARGE;
    return BFC_OK;
}

static int carve_batch(Carver &c, const bfc_graph *g, uint32_t nrep, const bfc_replica_info *info,
                       BatchWs &w) {
    BatchSizes z;
    BFC_TRY(batch_sizes(nrep, info, z));
    const uint64_t M = z.M;
    carve_filter(c, g, w.f);
    const uint64_t nv = (uint64_t)g->n_left > g->n_right ? g->n_left : g->n_right;
    w.ml = c.take<uint32_t>(pad64(g->n_left));
    w.mr = c.take<uint32_t>(pad64(g->n_right));
    w.scan_tmp_v = c.take<uint32_t>(scan_tmp_elems(nv));
    w.kl = c.take<uint32_t>(pad64(M));
    w.kr = c.take<uint32_t>(pad64(M));
    w.kept_dev = c.take<uint32_t>(nrep);
    w.sizes_dev = c.take<uint32_t>(2 * (uint64_t)nrep);
    w.part_l = c.take<uint32_t>(nrep + 1);
    w.part_r = c.take<uint32_t>(nrep + 1);
    w.div = c.take<double>(nrep);
    w.mul = c.take<double>(nrep);
    size_t sb, bb, ub, pb;
    BFC_TRY(bfc_graph_storage_size((uint32_t)z.NL, (uint32_t)z.NR, M, &sb));
    BFC_TRY(bfc_graph_build_ws_size((uint32_t)z.NL, (uint32_t)z.NR, M, &bb));
    // union workspace: offsets per part plus degree slots for both sides
    {
        Carver u(nullptr, 0);
        u.take<uint64_t>(3 * ((uint64_t)nrep + 1));
        u.take<uint32_t>(pad64(z.SL));
        u.take<uint32_t>(pad64(z.SR));
        u.take<uint32_t>(3 * ((uint64_t)nrep + 1));
        u.take<uint8_t>(nrep + 1);
        u.take<unsigned long long>(2 * (uint64_t)nrep);
        ub = u.used + 16 * 256;     // the union carves these in more, separately rounded pieces
    }
    {
        // bfc_exact_parts on a graph of these sizes, counted from L
        Carver e(nullptr, 0);
        e.take<char>(exact_ws_bound((uint32_t)z.NL, (uint32_t)z.NR, M));
        e.take<unsigned long long>(pad64(z.NL > z.NR ? z.NL : z.NR));
        e.take<unsigned long long>(1);
        pb = e.used;
    }
    w.storage_bytes = sb;
    w.storage = c.take<char>(sb);
    w.work_bytes = bb;
    if (ub > w.work_bytes) w.work_bytes = ub;
    if (pb > w.work_bytes) w.work_bytes = pb;
    w.work = c.take<char>(w.work_bytes);
    return BFC_OK;
}

}  // namespace bfc

extern "C" {

int bfc_spar_batch_filter_ws_size(const bfc_graph *g, uint32_t nrep, size_t *bytes) {
    if (!g || !bytes) return BFC_E_NULL;
    Carver c(nullptr, 0);
    FilterWs w;
    carve_filter(c, g, w);
    c.take<uint32_t>(pad64(g->n_left));
    c.take<uint32_t>(pad64(g->n_right));
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
    FilterWs w;
    carve_filter(c, g, w);
    uint32_t *deg_l = c.take<uint32_t>(pad64(g->n_left));
    uint32_t *deg_r = c.take<uint32_t>(pad64(g->n_right));
    unsigned long long *st = c.take<unsigned long long>(5 * (uint64_t)nrep);
    if (!c.fits()) return BFC_E_WS_SMALL;
    k_zero64<<<grid_for(5 * (uint64_t)nrep), 256, 0, s>>>(st, 5 * (uint64_t)nrep);
    unsigned gr = grid_for(g->n_left, 4);
    if (gr > 8192) gr = 8192;
    unsigned gl = grid_for(g->n_left), gR = grid_for(g->n_right);
    if (gl > 4096) gl = 4096;
    if (gR > 4096) gR = 4096;
    for (uint32_t i = 0; i < nrep; i++) {
        FilterArgs f;
        BFC_TRY(filter_replica(g, reps[i], w, f, s));
        unsigned long long *o = st + 5 * (uint64_t)i;
        k_store_last<<<1, 64, 0, s>>>(w.flag, g->n_edges, (uint32_t *)(o + 4));
        // the scan left the flags as running counts: recompute the flags for the degrees
        k_zero32<<<grid_for(g->n_left), 256, 0, s>>>(deg_l, g->n_left);
        k_zero32<<<grid_for(g->n_right), 256, 0, s>>>(deg_r, g->n_right);
        if (g->n_edges) {
            k_filter<<<gr, 256, 0, s>>>(f, w.flag);
            k_kept_degrees<<<gr, 256, 0, s>>>(f, w.flag, deg_l, deg_r);
        }
        if (g->n_left) k_deg_stats<<<gl, 256, 0, s>>>(deg_l, g->n_left, o);
        if (g->n_right) k_deg_stats<<<gR, 256, 0, s>>>(deg_r, g->n_right, o + 2);
        BFC_HIP(hipGetLastError());
    }
    std::vector<unsigned long long> h(5 * (size_t)nrep);
    BFC_HIP(hipMemcpyAsync(h.data(), st, h.size() * 8, hipMemcpyDeviceToHost, s));
    BFC_HIP(hipStreamSynchronize(s));
    for (uint32_t i = 0; i < nrep; i++) {
        const unsigned long long *o = &h[5 * (size_t)i];
        h_info[i].kept = (uint32_t)o[4];
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
    BFC_TRY(carve_batch(c, g, nrep, h_info, w));
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
    BFC_TRY(carve_batch(c, g, nrep, h_info, w));
    if (!c.fits()) return BFC_E_WS_SMALL;
    std::vector<uint64_t> h_kept(nrep);
    for (uint32_t i = 0; i < nrep; i++) h_kept[i] = h_info[i].kept;

    // 1. kept edges of every replica into the pool, vertices renumbered densely
    std::vector<uint64_t> eoff(nrep + 1, 0);
    for (uint32_t i = 0; i < nrep; i++) eoff[i + 1] = eoff[i] + h_kept[i];
    const unsigned gr = grid_for(g->n_left, 4) > 8192 ? 8192 : grid_for(g->n_left, 4);
    for (uint32_t i = 0; i < nrep; i++) {
        FilterArgs f;
        BFC_TRY(filter_replica(g, reps[i], w.f, f, s));
        uint32_t *kl = w.kl + eoff[i], *kr = w.kr + eoff[i];
        const uint64_t mk = h_kept[i];
        if (g->n_edges) {
            k_compact<<<gr, 256, 0, s>>>(f, w.f.flag, kl, kr, (uint32_t)mk);
            k_store_last<<<1, 64, 0, s>>>(w.f.flag, g->n_edges, w.kept_dev + i);
        } else {
            k_zero32<<<1, 64, 0, s>>>(w.kept_dev + i, 1);
        }
        k_zero32<<<grid_for(g->n_left), 256, 0, s>>>(w.ml, g->n_left);
        k_zero32<<<grid_for(g->n_right), 256, 0, s>>>(w.mr, g->n_right);
        if (mk) k_mark_ends<<<grid_for(mk), 256, 0, s>>>(kl, kr, mk, w.ml, w.mr);
        BFC_HIP(hipGetLastError());
        if (g->n_left) BFC_TRY(scan_u32_inclusive(w.ml, w.ml, g->n_left, w.scan_tmp_v, s));
        if (g->n_right) BFC_TRY(scan_u32_inclusive(w.mr, w.mr, g->n_right, w.scan_tmp_v, s));
        if (mk) k_renumber<<<grid_for(mk), 256, 0, s>>>(kl, kr, mk, w.ml, w.mr);
        k_store_last<<<1, 64, 0, s>>>(w.ml, g->n_left, w.sizes_dev + 2 * (uint64_t)i);
        k_store_last<<<1, 64, 0, s>>>(w.mr, g->n_right, w.sizes_dev + 2 * (uint64_t)i + 1);
        BFC_HIP(hipGetLastError());
    }
    std::vector<uint32_t> kept(nrep), sizes(2 * (size_t)nrep);
    BFC_HIP(hipMemcpyAsync(kept.data(), w.kept_dev, nrep * 4, hipMemcpyDeviceToHost, s));
    BFC_HIP(hipMemcpyAsync(sizes.data(), w.sizes_dev, sizes.size() * 4, hipMemcpyDeviceToHost, s));
    BFC_HIP(hipStreamSynchronize(s));
    for (uint32_t i = 0; i < nrep; i++)        // h_info must be this graph's phase 1
        if (kept[i] != h_kept[i] || sizes[2 * (size_t)i] != h_info[i].n_left ||
            sizes[2 * (size_t)i + 1] != h_info[i].n_right)
            return BFC_E_ARG;

    // 2. the union (parts oriented by ExactBFC's rule), its CSRs, one count
    std::vector<uint32_t> nl(nrep), nr(nrep), part_l(nrep + 1), part_r(nrep + 1);
    std::vector<uint8_t> swapped(nrep);
    for (uint32_t i = 0; i < nrep; i++) {
        nl[i] = sizes[2 * (size_t)i];
        nr[i] = sizes[2 * (size_t)i + 1];
    }
    BFC_TRY(bfc_batch_union(nrep, nl.data(), nr.data(), eoff.data(), w.kl, w.kr, w.kl, w.kr,
                            part_l.data(), part_r.data(), swapped.data(), w.work, w.work_bytes,
                            s));
    bfc_graph u;
    BFC_HIP(hipMemcpyAsync(w.part_l, part_l.data(), (nrep + 1) * 4, hipMemcpyHostToDevice, s));
    BFC_HIP(hipMemcpyAsync(w.part_r, part_r.data(), (nrep + 1) * 4, hipMemcpyHostToDevice, s));
    BFC_TRY(bfc_graph_build_parts(part_l[nrep], part_r[nrep], eoff[nrep], w.kl, w.kr, nrep,
                                  w.part_l, w.part_r, w.storage, w.storage_bytes, w.work,
                                  w.work_bytes, s, &u));
    BFC_TRY(bfc_exact_parts(&u, nrep, w.part_l, tuning, d_beta, w.work, w.work_bytes, s));

    // 3. estimates, in the single-replica expressions
    std::vector<double> div(nrep), mul(nrep);
    for (uint32_t i = 0; i < nrep; i++) {
        const bfc_replica &r = reps[i];
        if (r.kind == BFC_REPLICA_ESPAR) {
            div[i] = (r.p * r.p) * (r.p * r.p);
            mul[i] = 0.0;
        } else {
            const double N = (double)r.ncolors;
            div[i] = 0.0;
            mul[i] = N * N * N;
        }
    }
    BFC_HIP(hipMemcpyAsync(w.div, div.data(), nrep * 8, hipMemcpyHostToDevice, s));
    BFC_HIP(hipMemcpyAsync(w.mul, mul.data(), nrep * 8, hipMemcpyHostToDevice, s));
    k_est_batch<<<grid_for(nrep), 256, 0, s>>>((const unsigned long long *)d_beta, w.div, w.mul,
                                               nrep, d_est);
    BFC_HIP(hipGetLastError());
    BFC_HIP(hipStreamSynchronize(s));
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

// Weights, prefix sums and k draws over n items; returns BFC_E_PROBS for
// invalid probabilities (reads the check back: synchronises).
static int sample_draws(const double *d_probs, uint64_t n, uint64_t k, uint64_t seed,
                        uint32_t tag, SampWs &w, hipStream_t s) {
    BFC_HIP(hipMemsetAsync(w.flags, 0, sizeof(ProbFlags), s));
    if (d_probs) {
        k_prob_scan<<<grid_for(n), 256, 0, s>>>(d_probs, n, w.flags);
        ProbFlags hf;
        BFC_HIP(hipMemcpyAsync(&hf, w.flags, sizeof(hf), hipMemcpyDeviceToHost, s));
        BFC_HIP(hipStreamSynchronize(s));
        if (hf.bad || hf.max_bits == 0) return BFC_E_PROBS;
        k_quantise<<<grid_for(n), 256, 0, s>>>(d_probs, n, w.flags, w.w);
        BFC_HIP(hipMemcpyAsync(w.pre, w.w, n * sizeof(unsigned long long),
                               hipMemcpyDeviceToDevice, s));
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
    ProbFlags hf;
    BFC_HIP(hipMemcpyAsync(&hf, w.flags, sizeof(hf), hipMemcpyDeviceToHost, s));
    BFC_HIP(hipStreamSynchronize(s));
    return hf.overflow ? BFC_E_OVERFLOW_RISK : BFC_OK;
}

}  // namespace bfc

extern "C" {

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
    BFC_HIP(hipMemsetAsync(w.mark_l, 0, pad64(g->n_left), s));
    BFC_HIP(hipMemsetAsync(w.mark_r, 0, pad64(g->n_right), s));
    k_mark_vertices<<<grid_for(k), 256, 0, s>>>(k, w.draw, g->n_left, g->rank_l, g->rank_r,
                                                w.mark_l, w.mark_r, d_ids);
    BFC_HIP(hipMemsetAsync(w.cnt_l, 0, pad64(g->n_left) * 8, s));
    BFC_HIP(hipMemsetAsync(w.cnt_r, 0, pad64(g->n_right) * 8, s));
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
    BFC_HIP(hipMemsetAsync(mark, 0, pad64(nA), s));
    k_pos_of_edge<<<grid_for(m), 256, 0, s>>>(from_r ? g->eid_r : g->eid_l, m, w.pos);
    k_mark_edges<<<grid_for(k), 256, 0, s>>>(k, w.draw, w.pos, from_r ? g->off_r : g->off_l, nA,
                                             mark);
    BFC_HIP(hipMemsetAsync(w.cnt_e, 0, pad64(m) * 8, s));
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
    k_fast_total<<<1, 64, 0, s>>>(k, alpha, w.parts, d_est);
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
