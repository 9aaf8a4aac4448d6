/*
 * bfc.h -- butterfly counting in bipartite graphs on AMD Instinct MI355X
 * (gfx950).  C ABI of libbfc.so.
 *
 * Problem (Sec. 2 of Sanei-Mehri, Sariyuce, Tirthapura, "Butterfly Counting
 * in Bipartite Networks"): G = (L u R, E) is a simple bipartite graph.  A
 * butterfly is a 2x2 biclique {a,b} x {x,y}; B(G) is their number, B_v the
 * number containing vertex v, B_e the number containing edge e.
 *
 * Conventions for every call below.
 *  - Vertex ids are uint32, dense per side: 0 <= l < n_left, 0 <= r < n_right.
 *  - Every pointer named d_* is DEVICE memory owned by the caller (allocate it
 *    with hipMalloc, torch, ...).  The library never allocates device memory:
 *    scratch space is a caller workspace whose size a *_ws_size query gives.
 *    Workspaces and outputs must be 256-byte aligned.
 *  - Calls run asynchronously on the given stream unless stated otherwise; the
 *    caller synchronises before reading outputs.  Concurrent calls that share
 *    a workspace race.
 *  - Every call returns BFC_OK (0) or a negative BFC_E_* code and never throws
 *    across the ABI.  bfc_status_str() names a code; after BFC_E_HIP,
 *    bfc_last_hip_error() gives the HIP error string of the calling thread.
 *  - Integer counts are exact uint64.  Floating-point estimates are IEEE
 *    binary64 computed in a fixed order, so they are reproducible bit for bit.
 */
#ifndef BFC_H
#define BFC_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BFC_OK 0
#define BFC_E_NULL (-1)          /* a required pointer is NULL */
#define BFC_E_ARG (-2)           /* bad scalar argument (side, p, N, k, ...) */
#define BFC_E_ID_RANGE (-3)      /* an edge endpoint id >= its side's size */
#define BFC_E_DUP_EDGE (-4)      /* the edge list repeats an edge (not simple) */
#define BFC_E_TOO_LARGE (-5)     /* m >= 2^32 - 64 or a side >= 2^32 - 64 */
#define BFC_E_WS_SMALL (-6)      /* workspace or storage smaller than queried */
#define BFC_E_PROBS (-7)         /* probabilities negative, NaN, inf or all 0 */
#define BFC_E_OVERFLOW_RISK (-8) /* a uint64 count could overflow */
#define BFC_E_HIP (-9)           /* a HIP runtime call failed */
#define BFC_E_ALIGN (-10)        /* a device pointer is not 256-byte aligned */

#define BFC_SIDE_AUTO 0          /* the paper's rule (ExactBFC side choice) */
#define BFC_SIDE_L 1             /* start from L (midpoints in R) */
#define BFC_SIDE_R 2             /* start from R (midpoints in L) */

const char *bfc_status_str(int code);
const char *bfc_last_hip_error(void);

/* ---------------------------------------------------------------------- */
/* Graph: both adjacency structures (CSR) of G, built on the device.       */
/*                                                                          */
/* Each side's vertices are ranked by (degree ascending, id ascending); rows */
/* are stored in rank order and every adjacency list holds the ranks of the */
/* opposite side in ascending order.  The rank is the order "w precedes v"  */
/* of ExactBFC (Sec. 4): any strict total order counts every same-side pair */
/* once, and this one keeps the per-start work small.                       */
/*   off_x[i]..off_x[i+1]  row of the vertex of rank i on side x            */
/*   adj_x[k]              rank (opposite side) of the k-th neighbour        */
/*   eid_x[k]              index in the caller's edge list of that edge      */
/*   xpos_x[k]             position of the same edge in the other side's adj */
/*   rank_x[id], id_x[rank] the permutation between ids and ranks            */
/* All arrays live inside one caller-owned storage buffer.                   */
/* ---------------------------------------------------------------------- */
typedef struct bfc_graph {
    uint32_t n_left, n_right;
    uint64_t n_edges;
    const uint32_t *off_l, *adj_l, *eid_l, *xpos_l, *rank_l, *id_l;
    const uint32_t *off_r, *adj_r, *eid_r, *xpos_r, *rank_r, *id_r;
    /* statistics, host values filled by bfc_graph_build */
    uint64_t sumsq_l, sumsq_r;            /* sum of squared degrees per side */
    uint64_t wedges_mid_l, wedges_mid_r;  /* sum of C(d,2): wedges with that midpoint side */
    uint32_t max_deg_l, max_deg_r;
    int device;                           /* HIP device the arrays live on */
} bfc_graph;

/* Bytes of the storage buffer a graph of this size needs. */
int bfc_graph_storage_size(uint32_t n_left, uint32_t n_right, uint64_t n_edges, size_t *bytes);
/* Bytes of workspace bfc_graph_build needs (freed by the caller after). */
int bfc_graph_build_ws_size(uint32_t n_left, uint32_t n_right, uint64_t n_edges, size_t *bytes);

/* Build both CSRs from the caller's edge list d_l[i], d_r[i] (i < n_edges,
 * device uint32).  Validates the simple-graph assumption of Sec. 2:
 * BFC_E_ID_RANGE if an id is out of range, BFC_E_DUP_EDGE if an edge repeats.
 * SYNCHRONOUS: waits for the stream (it reads the statistics back).  The
 * graph stays valid while the storage buffer lives; the edge list and the
 * workspace may be freed after the call. */
int bfc_graph_build(uint32_t n_left, uint32_t n_right, uint64_t n_edges,
                    const uint32_t *d_l, const uint32_t *d_r,
                    void *d_storage, size_t storage_bytes,
                    void *d_ws, size_t ws_bytes, hipStream_t stream, bfc_graph *out);
/* The same for a disjoint union of nparts graphs whose vertices occupy id
 * ranges: part q owns the L ids [d_part_l[q], d_part_l[q + 1]) and the R ids
 * [d_part_r[q], d_part_r[q + 1]) (device, nparts + 1 uint32 each, from 0 to
 * n_left / n_right).  Vertices are ranked by (part, degree, id), another
 * strict total order, so each part's vertices hold consecutive ranks and a
 * start's counter windows stay inside its own part.  Same workspace sizes. */
int bfc_graph_build_parts(uint32_t n_left, uint32_t n_right, uint64_t n_edges,
                          const uint32_t *d_l, const uint32_t *d_r, uint32_t nparts,
                          const uint32_t *d_part_l, const uint32_t *d_part_r,
                          void *d_storage, size_t storage_bytes,
                          void *d_ws, size_t ws_bytes, hipStream_t stream, bfc_graph *out);

/* ---------------------------------------------------------------------- */
/* Exact count, ExactBFC (Sec. 4, Lemma 1 Eq. (3)/(4), Lemma 2).            */
/* Side choice (BFC_SIDE_AUTO): start from R when sum_L d^2 < sum_R d^2,     */
/* else from L.  For every start u, midpoint v in N(u) and endpoint w in     */
/* N(v) ranked above u, C_u[w] is incremented and B += C(C_u[w], 2).         */
/* ---------------------------------------------------------------------- */
/* Side that `side` resolves to (BFC_SIDE_L or BFC_SIDE_R), or a BFC_E_*. */
int bfc_side_used(const bfc_graph *g, int side);
/* Wedges the count visits from that side: sum over midpoints of C(d,2). */
int bfc_wedges(const bfc_graph *g, int side, uint64_t *wedges);
int bfc_exact_ws_size(const bfc_graph *g, int side, size_t *bytes);
/* Writes B(G) to *d_total (device uint64).  BFC_E_OVERFLOW_RISK if
 * wedges * (max start degree - 1) / 2 could exceed 2^64 - 1.
 * bfc_exact = bfc_exact_plan + bfc_exact_count. */
int bfc_exact(const bfc_graph *g, int side, uint64_t *d_total,
              void *d_ws, size_t ws_bytes, hipStream_t stream);
/* The two halves of bfc_exact.  The plan (per-call preparation of ExactBFC's
 * walk: adjacency segments at counter-window boundaries, per-start wedge
 * counts and the largest-first work queue) is written into the workspace;
 * bfc_exact_count launches the count itself and may be repeated on a
 * workspace planned for the same graph and side. */
int bfc_exact_plan(const bfc_graph *g, int side, void *d_ws, size_t ws_bytes,
                   hipStream_t stream);
int bfc_exact_count(const bfc_graph *g, int side, uint64_t *d_total,
                    void *d_ws, size_t ws_bytes, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): bfc_exact
 * with the same kernels and result, its workspace taken from a static device
 * array of BFC_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it
 * runs on until the process ends.  The call allocates nothing.  It runs on
 * the current device, asynchronously on `stream`.  BFC_E_TOO_LARGE when the
 * graph needs a larger workspace (bfc_exact_ws_size; 128 MiB holds graphs of
 * about 3.5 million edges).  Every call on one GPU shares that GPU's array:
 * calls that overlap on one GPU (other streams, other host threads) race, and
 * the caller must order them. */
#define BFC_NOALLOC_SCRATCH_BYTES (128u << 20)
int bfc_exact_noalloc(const bfc_graph *g, int side, uint64_t *d_total, hipStream_t stream);

/* ---------------------------------------------------------------------- */
/* Local counts (Sec. 2 definitions; Eq. (2); vBFC and eBFC of Sec. 4.2).   */
/*   B_v = sum over same-side w != v of C(|N(v) & N(w)|, 2)                 */
/*   B_(a,x) = sum over b in N(x), b != a of (|N(a) & N(b)| - 1)             */
/* Computed for every vertex / edge in one pass from the cheaper side.      */
/* Outputs are indexed by the caller's ids (d_cnt_l[n_left], d_cnt_r[n_right]) */
/* and edge order (d_cnt_e[n_edges]).  Any of the three may be NULL (not    */
/* wanted), but not all.                                                    */
/* ---------------------------------------------------------------------- */
int bfc_local_ws_size(const bfc_graph *g, size_t *bytes);
int bfc_local(const bfc_graph *g, uint64_t *d_cnt_l, uint64_t *d_cnt_r, uint64_t *d_cnt_e,
              void *d_ws, size_t ws_bytes, hipStream_t stream);
/* bfc_local with the part size of hub starts given: a start of more than
 * 255 midpoints whose walk visits t wedges is cut into ceil(t / split_wedges)
 * runs of counter windows (at most one per window, at most 4096), each
 * walked by its own workgroup; the parts add into the start's counts and the
 * last part to finish writes its edges.  split_wedges = 0: the default of
 * bfc_local, 2^24.  Same results for any value. */
int bfc_local_split_ws_size(const bfc_graph *g, uint64_t split_wedges, size_t *bytes);
int bfc_local_split(const bfc_graph *g, uint64_t split_wedges, uint64_t *d_cnt_l,
                    uint64_t *d_cnt_r, uint64_t *d_cnt_e, void *d_ws, size_t ws_bytes,
                    hipStream_t stream);
int bfc_per_vertex(const bfc_graph *g, uint64_t *d_cnt_l, uint64_t *d_cnt_r,
                   void *d_ws, size_t ws_bytes, hipStream_t stream);
int bfc_per_edge(const bfc_graph *g, uint64_t *d_cnt_e, void *d_ws, size_t ws_bytes,
                 hipStream_t stream);

/* ---------------------------------------------------------------------- */
/* Estimators.  Random decisions use Philox-4x32-10 (Salmon et al., SC'11)  */
/* keyed by `seed`, with one fixed counter per decision, so a result does   */
/* not depend on thread order and is reproducible bit for bit:             */
/*   ESpar keep of edge (l, r): counter (l, r, 0x45535052, 0), x = out0 |   */
/*     out1 << 32, kept iff x < floor(p * 2^64) (p = 1 keeps every edge);   */
/*   ClrSpar colour of vertex v of side s (0 = L, 1 = R): counter (v, s,    */
/*     0x434C5253, attempt), x = out0, retried while x >= 2^32 - 2^32 mod N, */
/*     colour = x mod N;                                                     */
/*   draw i of VSamp / ESamp: counter (i & 0xffffffff, i >> 32, 0x56445257  */
/*     / 0x45445257, attempt), x = out0 | out1 << 32, retried while          */
/*     x >= 2^64 - 2^64 mod n, value x mod n.                                */
/* Weighted draws (d_probs given) quantise the probabilities to integer     */
/* weights q_j = p_j > 0 ? max(1, floor(p_j / max(p) * (2^32 - 1))) : 0 and  */
/* take the first j whose inclusive prefix sum of q exceeds a draw below    */
/* Q = sum(q).  These calls only launch kernels (asynchronous, capturable   */
/* into a HIP graph): probabilities that are negative, NaN, infinite or all */
/* zero are detected on the device and make the estimate NaN (the draws     */
/* then use equal weights); bfc_probs_check reports them to the host.       */
/* ---------------------------------------------------------------------- */
/* Synchronous check of probabilities for the weighted samplers: BFC_OK, or
 * BFC_E_PROBS when one is negative, NaN or infinite or all are 0.  d_ws:
 * bfc_probs_check_ws_size bytes. */
int bfc_probs_check_ws_size(size_t *bytes);
int bfc_probs_check(const double *d_probs, uint64_t n, void *d_ws, size_t ws_bytes,
                    hipStream_t stream);
/* The sparsifiers build the kept graph on the device without sorting (each
 * CSR row filtered in order, the vertices that keep an edge renumbered in
 * rank order: another strict total order, so the count is unchanged), lay it
 * out on the graph's own sizes (the kept sizes never leave the device) and
 * count it from the side ExactBFC's rule picks for the graph itself (the
 * count is the same from either side).  Asynchronous: kernels only. */
int bfc_spar_ws_size(const bfc_graph *g, size_t *bytes);
/* ESpar (Sec. 6.1): keep each edge with probability p in (0, 1], count the
 * kept graph's butterflies beta exactly, estimate = beta / ((p*p)*(p*p)).
 * *d_kept_bflies = beta, *d_est = estimate, *d_kept_edges (may be NULL) =
 * number of kept edges (device uint64 / double / uint64).  BFC_E_ARG unless
 * 0 < p <= 1. */
int bfc_espar(const bfc_graph *g, double p, uint64_t seed, uint64_t *d_kept_bflies,
              double *d_est, uint64_t *d_kept_edges, void *d_ws, size_t ws_bytes,
              hipStream_t stream);
/* ClrSpar (Sec. 6.2): colour the vertices with ncolors >= 1 colours, keep the
 * monochromatic edges, count their butterflies beta exactly, estimate =
 * beta * (N * N * N) in binary64; outputs as bfc_espar.  BFC_E_ARG if
 * ncolors == 0. */
int bfc_clrspar(const bfc_graph *g, uint32_t ncolors, uint64_t seed, uint64_t *d_mono_bflies,
                double *d_est, uint64_t *d_kept_edges, void *d_ws, size_t ws_bytes,
                hipStream_t stream);

/* VSamp (Sec. 5.1): k >= 1 draws with replacement of a vertex, uniformly or
 * by d_probs (n_left + n_right doubles: L ids then R ids).  d_ids[i] is the
 * drawn vertex (global id: L id, or n_left + R id), d_counts[i] its count B_v
 * (vBFC).  *d_est: uniform: (double)sum(counts) * n / (4 k) with the sum exact
 * in uint64 (the mean of Alg. VSamp over k draws); weighted: the
 * Hansen-Hurwitz mean of B_v * Q / (4 q_v), summed left to right in blocks of
 * 1024 draws and the block sums left to right.  *d_est is NaN for invalid
 * probabilities and when the exact uniform sum would overflow 64 bits. */
int bfc_vsamp_ws_size(const bfc_graph *g, uint64_t k, size_t *bytes);
int bfc_vsamp(const bfc_graph *g, const double *d_probs, uint64_t k, uint64_t seed,
              uint32_t *d_ids, uint64_t *d_counts, double *d_est, void *d_ws, size_t ws_bytes,
              hipStream_t stream);
/* The draws of bfc_vsamp alone, without counting: for the same graph,
 * probabilities, k and seed, d_ids equals bfc_vsamp's.  d_weights (k uint32,
 * may be NULL) receives each draw's integer weight w_v (1 when d_probs is
 * NULL) and *d_total_weight (device uint64, may be NULL) the sum of all
 * weights Q (n when uniform), so that with known counts B_v the estimate
 * can be formed exactly as bfc_vsamp forms it.  Invalid probabilities give
 * equal weights (check them with bfc_probs_check). */
int bfc_vsamp_draws_ws_size(const bfc_graph *g, uint64_t k, size_t *bytes);
int bfc_vsamp_draws(const bfc_graph *g, const double *d_probs, uint64_t k, uint64_t seed,
                    uint32_t *d_ids, uint32_t *d_weights, uint64_t *d_total_weight, void *d_ws,
                    size_t ws_bytes, hipStream_t stream);
/* ESamp (Sec. 5.2): the same over edges (d_probs: n_edges doubles in the
 * caller's edge order); d_eids[i] the drawn edge's index, d_counts[i] its B_e
 * (eBFC), estimate with n = n_edges. */
int bfc_esamp_ws_size(const bfc_graph *g, uint64_t k, size_t *bytes);
int bfc_esamp(const bfc_graph *g, const double *d_probs, uint64_t k, uint64_t seed,
              uint64_t *d_eids, uint64_t *d_counts, double *d_est, void *d_ws, size_t ws_bytes,
              hipStream_t stream);
/* ESamp with Fast-eBFC (Sec. 5.5): the edges are drawn exactly as bfc_esamp
 * draws them (same seed: same d_eids), but each drawn edge's count is
 * estimated, not counted.  Draw i (k < 2^32) runs alpha >= 1 trials on its
 * edge e = (a, x): trial j picks a neighbour b of x and a neighbour y of a
 * uniformly (one Philox block at counter (i, j, 'FEBC', attempt), words
 * 0-1 for b and 2-3 for y, both by rejection; neighbours in ascending rank
 * order) and hits iff b != a, y != x and (b, y) is an edge.  Exactly B_e of
 * the d_a * d_x picks hit, so hits * d_a * d_x / alpha is an unbiased
 * estimate of B_e (the lemma of Sec. 5.5).
 * d_eids[i] (uint64): the drawn edge's index in the caller's edge list;
 * d_hits[i] (uint32): its number of hits; *d_est: term_i = ((double)hits_i
 * * (double)(d_a * d_x)) * s_i with s_i = (double)m / 4 (uniform) or
 * Q / (4.0 * q_i) (weighted, as bfc_esamp), summed left to right within
 * blocks of 1024 draws, block sums left to right, divided by
 * ((double)k * (double)alpha).  BFC_E_ARG for k == 0, k >= 2^32 or
 * alpha == 0; NaN estimate for invalid probabilities, as bfc_esamp. */
int bfc_esamp_fast_ws_size(const bfc_graph *g, uint64_t k, size_t *bytes);
int bfc_esamp_fast(const bfc_graph *g, const double *d_probs, uint64_t k, uint32_t alpha,
                   uint64_t seed, uint64_t *d_eids, uint32_t *d_hits, double *d_est,
                   void *d_ws, size_t ws_bytes, hipStream_t stream);

/* WSamp (Sec. 5.3): k < 2^32 draws with replacement of a uniform wedge, each
 * counted exactly.  Wedges are numbered 0 .. W-1 (W = wedges_mid_l +
 * wedges_mid_r): vertices in global order (L ids, then n_left + R id) own
 * consecutive ranges of C(d,2) numbers, and number p of vertex u's range is
 * the pair of positions (j1, j2), j1 < j2, p = C(j2,2) + j1, in u's
 * neighbour list (ascending rank order).  Draw i takes a uniform number
 * below W from the Philox stream (i lo, i hi, 'WDRW', attempt) by
 * rejection.  d_mids[i] (uint32): the midpoint (global id); d_ends[2i],
 * d_ends[2i+1] (uint32): the endpoints j1 and j2 (global ids); d_counts[i]
 * (uint64): butterflies through the wedge, |G_v n G_w| - 1; *d_est =
 * ((double)sum(counts) * (double)W) / (4.0 * (double)k), the sum exact in
 * uint64.  BFC_E_ARG for k == 0, k >= 2^32 or a graph without wedges.
 * Asynchronous. */
int bfc_wsamp_ws_size(const bfc_graph *g, uint64_t k, size_t *bytes);
int bfc_wsamp(const bfc_graph *g, uint64_t k, uint64_t seed, uint32_t *d_mids, uint32_t *d_ends,
              uint64_t *d_counts, double *d_est, void *d_ws, size_t ws_bytes,
              hipStream_t stream);

/* (eps, delta) estimates from the sparsifiers (Sec. 6.1, 6.2).
 * bfc_spar_threshold (host): the sampling rate of the ESpar lemma,
 * p = min(1, max((24/B)^(1/4), sqrt(24 D / B), 24 D^2 / B)), or for ClrSpar
 * the largest number of colours N with 1/N > max((32/B)^(1/3),
 * sqrt(32 D / B), 32 D^2 / B) (at least 1; *p = 1/N), from an estimate B of
 * the count (a pilot, e.g. bfc_esamp_fast) and the largest degree D.
 * kind: BFC_REPLICA_ESPAR or BFC_REPLICA_CLRSPAR.  B <= 0 keeps everything.
 * bfc_eps_delta_plan (host): g groups of r estimates, r = ceil(3 / (2
 * eps^2)), g = ceil(8 ln(1/delta)) made odd.  Above the thresholds one
 * estimate's variance is below 3 B^2 / 8 (the lemmas' argument with
 * butterfly pairs counted in both orders and per-butterfly pair bounds), so
 * a group mean misses B by more than eps B with probability at most 1/4
 * (Chebyshev) and the median of the g means with probability at most
 * exp(-g/8) <= delta (Hoeffding).  BFC_E_ARG unless 0 < eps <= 1,
 * 0 < delta < 1 and g <= 4096.
 * bfc_median_of_means (device): d_x holds groups * per_group doubles, group
 * q at [q r, q r + r); d_means[q] = (sum left to right) / r; *d_median = the
 * mean at sorted position (g - 1) / 2.  Asynchronous. */
int bfc_spar_threshold(int kind, double B, uint32_t max_deg, double *p, uint32_t *ncolors);
int bfc_eps_delta_plan(double eps, double delta, uint32_t *groups, uint32_t *per_group);
int bfc_median_of_means(const double *d_x, uint32_t groups, uint32_t per_group, double *d_means,
                        double *d_median, hipStream_t stream);

/* ---------------------------------------------------------------------- */
/* Batched exact counts: many graphs counted in one persistent launch.      */
/*                                                                          */
/* A batch is one disjoint union of parts, each oriented so that its start  */
/* side (ExactBFC's side choice, Sec. 4, applied per part) is the union's L; */
/* bfc_batch_union builds the union's edge list, bfc_graph_build its CSRs,  */
/* and bfc_exact_parts counts every part with one plan and one launch per   */
/* kernel class, returning each part's total.  Nothing here changes a      */
/* count: a part's total equals bfc_exact on that graph alone.              */
/* ---------------------------------------------------------------------- */
/* Launch shape of the count kernels; 0 in a field means its default.      */
typedef struct bfc_tuning {
    uint32_t narrow_max;          /* starts of degree <= this take the one-wave kernel (1..255; 255) */
    uint32_t chunk;               /* narrow starts taken from the queue at once (1..64; 4) */
    uint32_t narrow_waves_per_cu; /* narrow grid, waves per compute unit (1..8; 8) */
    uint32_t wide_groups_per_cu;  /* wide grid, workgroups per compute unit (1..2; 2) */
    uint32_t hash_small_max;      /* narrow starts with at most this many wedges use the
                                     one-wave hash table (1..2048; 1024; BFC_HASH_OFF: none) */
    uint32_t hash_mid_max;        /* ... else at most this many the four-wave one
                                     (1..16384; 16384; BFC_HASH_OFF: none) */
    uint32_t hash_passes;         /* passes of a hash start over its wedges (1..4; 0: as many
                                     as half-full tables need).  A pass that fills its
                                     table hands the start to the narrow window walk */
    uint32_t hash_max_density;    /* a start takes a hash table only when it has at most
                                     this many wedges per counter window its end points
                                     span (32) */
} bfc_tuning;
#define BFC_HASH_OFF 0xFFFFFFFFu

/* bfc_exact with a given launch shape (NULL: defaults); same result. */
int bfc_exact_tuned(const bfc_graph *g, int side, const bfc_tuning *tuning, uint64_t *d_total,
                    void *d_ws, size_t ws_bytes, hipStream_t stream);

/* Per-part totals of a disjoint union counted from L.  d_part_l (device,
 * nparts + 1 uint32, ascending): part q owns the L ids [d_part_l[q],
 * d_part_l[q + 1]) and the caller guarantees that its edges stay inside the
 * part.  d_totals (device, nparts uint64) receives each part's butterflies,
 * summed in a fixed order.  Asynchronous (plan, count, sums: kernels only),
 * so it may be captured into a HIP graph and replayed. */
int bfc_exact_parts_ws_size(const bfc_graph *g, size_t *bytes);
int bfc_exact_parts(const bfc_graph *g, uint32_t nparts, const uint32_t *d_part_l,
                    const bfc_tuning *tuning, uint64_t *d_totals, void *d_ws, size_t ws_bytes,
                    hipStream_t stream);

/* Autotuner: times candidate launch shapes of bfc_exact_tuned (nparts == 0,
 * automatic side; d_totals needs one uint64) or of bfc_exact_parts on this
 * batch, with events on the stream, and returns the fastest in *best (and
 * its time in *best_ms).  Synchronous; not for use under stream capture. */
int bfc_autotune_ws_size(const bfc_graph *g, size_t *bytes);
int bfc_autotune(const bfc_graph *g, uint32_t nparts, const uint32_t *d_part_l,
                 uint64_t *d_totals, void *d_ws, size_t ws_bytes, hipStream_t stream,
                 bfc_tuning *best, float *best_ms);

/* Union of ng graphs.  Graph q has h_nl[q] x h_nr[q] vertices and the edges
 * [h_eoff[q], h_eoff[q + 1]) of the concatenated device lists d_l, d_r (ids
 * local to the graph).  Each graph starts from R iff its sum of squared L
 * degrees is below its sum of squared R degrees (ExactBFC's rule); such a
 * graph is entered with its sides exchanged (h_swapped[q] = 1).  Writes the
 * union ids d_ul, d_ur (device, h_eoff[ng] each) and the host offsets
 * h_part_l / h_part_r (ng + 1): union L ids of graph q are [h_part_l[q],
 * h_part_l[q + 1]).  Synchronous.  Errors: BFC_E_ID_RANGE (a local id out of
 * range), BFC_E_TOO_LARGE (union sides beyond 2^32 - 1 vertices). */
int bfc_batch_union_ws_size(uint32_t ng, const uint32_t *h_nl, const uint32_t *h_nr,
                            const uint64_t *h_eoff, size_t *bytes);
int bfc_batch_union(uint32_t ng, const uint32_t *h_nl, const uint32_t *h_nr,
                    const uint64_t *h_eoff, const uint32_t *d_l, const uint32_t *d_r,
                    uint32_t *d_ul, uint32_t *d_ur, uint32_t *h_part_l, uint32_t *h_part_r,
                    uint8_t *h_swapped, void *d_ws, size_t ws_bytes, hipStream_t stream);

/* Replica batches: many ESpar / ClrSpar replicas of one graph counted in   */
/* one launch.  Each replica keeps the edges its single call would keep     */
/* (same parameters, same seed, same random stream), its kept graph becomes */
/* one part of a disjoint union (vertices without a kept edge dropped, the  */
/* others renumbered in rank order, oriented by ExactBFC's side rule on its */
/* own degrees), built without sorting, and bfc_exact_parts counts all      */
/* parts.  d_beta[i] and d_est[i] equal what bfc_espar / bfc_clrspar return */
/* for replica i, bit for bit.                                              */
#define BFC_REPLICA_ESPAR 0
#define BFC_REPLICA_CLRSPAR 1
typedef struct bfc_replica {
    uint32_t kind;      /* BFC_REPLICA_ESPAR or BFC_REPLICA_CLRSPAR */
    uint32_t ncolors;   /* ClrSpar: N >= 1 colours */
    double p;           /* ESpar: keep probability, 0 < p <= 1 */
    uint64_t seed;
} bfc_replica;
/* What phase 1 learns of each replica's kept graph (host). */
typedef struct bfc_replica_info {
    uint64_t kept;                        /* kept edges */
    uint32_t n_left, n_right;             /* vertices with a kept edge, per side */
    uint64_t sumsq_left, sumsq_right;     /* sums of squared kept degrees */
} bfc_replica_info;
/* Phase 1 (synchronous): h_info (host, nrep) for every replica. */
int bfc_spar_batch_filter_ws_size(const bfc_graph *g, uint32_t nrep, size_t *bytes);
int bfc_spar_batch_filter(const bfc_graph *g, uint32_t nrep, const bfc_replica *reps,
                          bfc_replica_info *h_info, void *d_ws, size_t ws_bytes,
                          hipStream_t stream);
/* Phase 2: the batch itself, laid out and its workspace sized from h_info,
 * which must be phase 1's output for the same graph and replicas.  Kernels
 * only (asynchronous), so it can be captured into a HIP graph and replayed.
 * On the device each replica's kept sizes are checked against h_info; if one
 * differs, nothing is written outside the workspace and every d_beta[i] is
 * 2^64 - 1 and every d_est[i] NaN.  d_beta (nrep uint64) and d_est (nrep
 * double) are device arrays.  BFC_E_TOO_LARGE when the union would exceed
 * 32-bit ids. */
int bfc_spar_batch_ws_size(const bfc_graph *g, uint32_t nrep, const bfc_replica *reps,
                           const bfc_replica_info *h_info, size_t *bytes);
int bfc_spar_batch(const bfc_graph *g, uint32_t nrep, const bfc_replica *reps,
                   const bfc_replica_info *h_info, const bfc_tuning *tuning, uint64_t *d_beta,
                   double *d_est, void *d_ws, size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------------------- */
/* Learned importance sampling (an addition to the paper's VSamp): a small  */
/* MLP predicts log1p(B_v) from per-vertex features; its predictions give   */
/* bfc_vsamp's probabilities.  It never changes a count.                    */
/*   parameters: bfc_mlp_param_count() floats, layout W1[8][64], b1[64],     */
/*   W2[64][64], b2[64], w3[64], b3 (FP32 master copy; device, caller-owned); */
/*   BF16 copy: the same count of uint16 at the same offsets (W1, W2, w3 are */
/*   read from it).  Layers: h1 = relu(x W1 + b1), h2 = relu(h1 W2 + b2),     */
/*   y = h2 w3 + b3, on the matrix cores in BF16 with FP32 accumulation; h1  */
/*   is rounded to BF16 before layer 2.                                      */
/* ---------------------------------------------------------------------- */
int bfc_mlp_param_count(void);
/* 8 BF16 features per vertex, rows by global id (L ids, then n_left + R id):
 * side, log1p d, log1p sum d_u, log1p sum d_u^2, log1p max d_u,
 * log1p sum(d_u - 1), log1p C(d,2), log1p(sum d_u / d) over the neighbours u,
 * each log term divided by 8.  d_feat: (n_left + n_right) * 8 uint16. */
int bfc_features(const bfc_graph *g, uint16_t *d_feat, hipStream_t stream);
/* BF16 copy of the FP32 parameters (round to nearest even). */
int bfc_mlp_bf16(const float *d_params, uint16_t *d_wbf16, hipStream_t stream);
/* y[r] for rows r < rows of d_x (rows * 8 BF16). */
int bfc_mlp_forward(const uint16_t *d_x, uint32_t rows, const float *d_params,
                    const uint16_t *d_wbf16, float *d_y, hipStream_t stream);
/* Training targets log1p(count) / 8 (FP32) from n uint64 per-vertex counts. */
int bfc_mlp_targets(const uint64_t *d_counts, uint64_t n, float *d_target, hipStream_t stream);
/* Mini-batch of `rows` (>= 1) rows; row r is feature row d_idx[r] with target
 * d_target[d_idx[r]] (d_idx NULL: row r itself).  Writes the gradient of
 * sum_r (y_r - t_r)^2 / rows with respect to every parameter into d_grad
 * (param_count floats, overwritten) and sum_r (y_r - t_r)^2 into *d_loss.
 * dZ2 and dZ1 are rounded to BF16 before the matrix-core products that use
 * them.  Per-wave partial sums go to the workspace (bfc_mlp_grad_ws_size
 * bytes) and are reduced in a fixed order, so results are reproducible. */
int bfc_mlp_grad_ws_size(uint32_t rows, size_t *bytes);
int bfc_mlp_grad(const uint16_t *d_x, const float *d_target, const uint32_t *d_idx,
                 uint32_t rows, const float *d_params, const uint16_t *d_wbf16, float *d_grad,
                 float *d_loss, void *d_ws, size_t ws_bytes, hipStream_t stream);
/* One Adam step (moments d_m1, d_m2; step >= 1 for the bias correction) on
 * the FP32 parameters, then the BF16 copy is refreshed. */
int bfc_adam_step(float *d_params, float *d_m1, float *d_m2, const float *d_grad,
                  uint16_t *d_wbf16, float lr, float beta1, float beta2, float eps,
                  uint32_t step, hipStream_t stream);
/* Probabilities for bfc_vsamp from predictions y (n floats, predicting
 * log1p(B_v)/8): p_v = max(expm1(8 y_v), floor_frac * mean_v expm1(8 y_v)^+),
 * the mean reduced in a fixed order; *d_mean (may be NULL) gets the mean.
 * floor_frac must be positive and finite (else BFC_E_ARG), so every p_v > 0
 * and the weighted VSamp estimate is unbiased for any predictions; when no
 * prediction is positive (mean 0) every p_v = 1 (uniform sampling). */
int bfc_probs_ws_size(size_t *bytes);
int bfc_probs_from_predictions(const float *d_y, uint64_t n, double floor_frac, double *d_probs,
                               double *d_mean, void *d_ws, size_t ws_bytes, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* BFC_H */
