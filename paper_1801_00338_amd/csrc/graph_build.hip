// Graph construction: both CSRs of a simple bipartite graph, in degree-rank
// order, from a caller edge list on the device.  Also the library's status
// strings and the uint32 prefix scan used by the planning kernels.
#include <cstring>
#include <rocprim/rocprim.hpp>

#include "common.h"

namespace bfc {

static thread_local char g_hip_err[256] = "";

void set_hip_error(hipError_t e) {
    const char *s = hipGetErrorString(e);
    strncpy(g_hip_err, s ? s : "unknown HIP error", sizeof(g_hip_err) - 1);
    g_hip_err[sizeof(g_hip_err) - 1] = 0;
}

int device_cu_count(int device) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
        n <= 0)
        n = 256;
    return n;
}

// ------------------------------------------------------------------ scan
// Reduce-then-scan over tiles of 4096 values: per-tile sums, an exclusive
// scan of the tile sums (one workgroup, serial over chunks of 1024), then a
// per-tile scan that adds its tile offset.
constexpr int SCAN_NT = 256;
constexpr int SCAN_PER = 16;
constexpr int SCAN_TILE = SCAN_NT * SCAN_PER;

size_t scan_tmp_elems(uint64_t n) { return (size_t)((n + SCAN_TILE - 1) / SCAN_TILE) + 64; }

__global__ __launch_bounds__(SCAN_NT) void k_scan_tile_sums(const uint32_t *in, uint64_t n,
                                                            uint32_t *sums) {
    __shared__ unsigned long long red[SCAN_NT / WAVE];
    uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE;
    unsigned long long s = 0;
    for (int i = 0; i < SCAN_PER; i++) {
        uint64_t idx = base + (uint64_t)i * SCAN_NT + threadIdx.x;
        if (idx < n) s += in[idx];
    }
    s = block_sum64<SCAN_NT>(s, red);
    if (threadIdx.x == 0) sums[blockIdx.x] = (uint32_t)s;
}

__global__ __launch_bounds__(1024) void k_scan_sums(uint32_t *sums, uint32_t nt) {
    __shared__ uint32_t red[1024 / WAVE + 1];
    uint32_t carry = 0;
    for (uint32_t b = 0; b < nt; b += 1024) {
        uint32_t i = b + threadIdx.x;
        uint32_t v = i < nt ? sums[i] : 0;
        uint32_t tot;
        uint32_t ex = block_excl_scan<1024>(v, red, &tot);
        if (i < nt) sums[i] = carry + ex;
        carry += tot;
    }
}

__global__ __launch_bounds__(SCAN_NT) void k_scan_tiles(const uint32_t *in, uint32_t *out,
                                                        uint64_t n, const uint32_t *offs) {
    __shared__ uint32_t red[SCAN_NT / WAVE + 1];
    uint64_t base = (uint64_t)blockIdx.x * SCAN_TILE + (uint64_t)threadIdx.x * SCAN_PER;
    uint32_t v[SCAN_PER];
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < SCAN_PER; i++) {
        uint64_t idx = base + i;
        v[i] = idx < n ? in[idx] : 0;
        s += v[i];
    }
    uint32_t tot;
    uint32_t ex = block_excl_scan<SCAN_NT>(s, red, &tot) + offs[blockIdx.x];
#pragma unroll
    for (int i = 0; i < SCAN_PER; i++) {
        uint64_t idx = base + i;
        ex += v[i];
        if (idx < n) out[idx] = ex;
    }
}

int scan_u32_inclusive(const uint32_t *in, uint32_t *out, uint64_t n, uint32_t *tmp,
                       hipStream_t s) {
    if (n == 0) return BFC_OK;
    uint32_t nt = (uint32_t)((n + SCAN_TILE - 1) / SCAN_TILE);
    k_scan_tile_sums<<<nt, SCAN_NT, 0, s>>>(in, n, tmp);
    k_scan_sums<<<1, 1024, 0, s>>>(tmp, nt);
    k_scan_tiles<<<nt, SCAN_NT, 0, s>>>(in, out, n, tmp);
    BFC_HIP(hipGetLastError());
    return BFC_OK;
}

// ------------------------------------------------------------------ build kernels
struct BuildFlags {
    uint32_t bad_id;
    uint32_t dup;
    uint32_t max_deg_l, max_deg_r;
    unsigned long long sumsq_l, sumsq_r, w_l, w_r;
};

__global__ void k_fill_u32(uint32_t *p, uint64_t n, uint32_t v) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_validate(const uint32_t *l, const uint32_t *r, uint64_t m, uint32_t nl,
                           uint32_t nr, BuildFlags *f) {
    bool bad = false;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < m;
         i += (uint64_t)gridDim.x * blockDim.x)
        bad |= (l[i] >= nl) | (r[i] >= nr);
    if (bad) atomicOr(&f->bad_id, 1u);
}

__global__ void k_degrees(const uint32_t *l, const uint32_t *r, uint64_t m, uint32_t *dl,
                          uint32_t *dr) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < m;
         i += (uint64_t)gridDim.x * blockDim.x) {
        atomicAdd(&dl[l[i]], 1u);
        atomicAdd(&dr[r[i]], 1u);
    }
}

__global__ void k_iota(uint32_t *p, uint32_t n) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = i;
}

// Keys (part, degree) for a part-major rank order: part q owns the ids
// [part[q], part[q + 1]).
__global__ void k_part_keys(const uint32_t *deg, uint32_t n, const uint32_t *part, uint32_t np,
                            unsigned long long *keys) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t lo = 0, hi = np;               // last q with part[q] <= i
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (part[mid] <= i) lo = mid; else hi = mid;
        }
        keys[i] = ((unsigned long long)lo << 32) | deg[i];
    }
}

__global__ void k_low_words(const unsigned long long *keys, uint32_t n, uint32_t *low) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        low[i] = (uint32_t)keys[i];
}

// After sorting (degree, id) pairs: rank[id_sorted[i]] = i; the sorted
// degrees become the row lengths in rank order (copied into off[1..n]).
__global__ void k_ranks(const uint32_t *ids_sorted, const uint32_t *deg_sorted, uint32_t n,
                        uint32_t *rank, uint32_t *row_len) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        rank[ids_sorted[i]] = i;
        row_len[i] = deg_sorted[i];
    }
}

__global__ void k_degree_stats(const uint32_t *deg, uint32_t n, unsigned long long *sumsq,
                               unsigned long long *wedges, uint32_t *maxdeg) {
    __shared__ unsigned long long red[256 / WAVE];
    unsigned long long s = 0, w = 0;
    uint32_t mx = 0;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        unsigned long long d = deg[i];
        s += d * d;
        w += d * (d - (d > 0)) / 2;
        mx = max(mx, (uint32_t)d);
    }
    s = block_sum64<256>(s, red);
    w = block_sum64<256>(w, red);
    if (threadIdx.x == 0) {
        atomicAdd(sumsq, s);
        atomicAdd(wedges, w);
    }
    mx = wave_min(~mx);
    if ((threadIdx.x & (WAVE - 1)) == 0) atomicMax(maxdeg, ~mx);
}

// Keys for one CSR: row rank in the high bits, column rank in the low bits.
__global__ void k_make_keys(const uint32_t *src, const uint32_t *dst, uint64_t m,
                            const uint32_t *rank_src, const uint32_t *rank_dst, int col_bits,
                            unsigned long long *keys, uint32_t *vals) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < m;
         i += (uint64_t)gridDim.x * blockDim.x) {
        keys[i] = ((unsigned long long)rank_src[src[i]] << col_bits) | rank_dst[dst[i]];
        vals[i] = (uint32_t)i;
    }
}

__global__ void k_unpack_keys(const unsigned long long *keys, uint64_t m, uint32_t col_mask,
                              uint32_t *adj, BuildFlags *f) {
    bool dup = false;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < m;
         i += (uint64_t)gridDim.x * blockDim.x) {
        unsigned long long k = keys[i];
        adj[i] = (uint32_t)k & col_mask;
        if (i > 0 && keys[i - 1] == k) dup = true;
    }
    if (dup) atomicOr(&f->dup, 1u);
}

// pos_of_edge[eid[k]] = k
__global__ void k_scatter_pos(const uint32_t *eid, uint64_t m, uint32_t *pos) {
    for (uint64_t k = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; k < m;
         k += (uint64_t)gridDim.x * blockDim.x)
        pos[eid[k]] = (uint32_t)k;
}

__global__ void k_gather_pos(const uint32_t *eid, uint64_t m, const uint32_t *pos, uint32_t *x) {
    for (uint64_t k = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; k < m;
         k += (uint64_t)gridDim.x * blockDim.x)
        x[k] = pos[eid[k]];
}

static inline int bits_for(uint32_t n) {
    int b = 1;
    while (b < 32 && (1ull << b) < (uint64_t)n) b++;
    return b;
}

static inline unsigned grid_for(uint64_t n, int nt = 256) {
    uint64_t g = (n + nt - 1) / nt;
    if (g < 1) g = 1;
    if (g > 65535ull * 16) g = 65535ull * 16;
    return (unsigned)g;
}

// Storage layout (uint32 arrays, each padded to a multiple of 64 entries).
struct Layout {
    uint32_t *off_l, *adj_l, *eid_l, *xpos_l, *rank_l, *id_l;
    uint32_t *off_r, *adj_r, *eid_r, *xpos_r, *rank_r, *id_r;
};

static Layout carve_storage(Carver &c, uint32_t nl, uint32_t nr, uint64_t m) {
    Layout L;
    L.off_l = c.take<uint32_t>(pad64(nl + 1ull));
    L.adj_l = c.take<uint32_t>(pad64(m + ADJ_SLACK));
    L.eid_l = c.take<uint32_t>(pad64(m));
    L.xpos_l = c.take<uint32_t>(pad64(m));
    L.rank_l = c.take<uint32_t>(pad64(nl));
    L.id_l = c.take<uint32_t>(pad64(nl));
    L.off_r = c.take<uint32_t>(pad64(nr + 1ull));
    L.adj_r = c.take<uint32_t>(pad64(m + ADJ_SLACK));
    L.eid_r = c.take<uint32_t>(pad64(m));
    L.xpos_r = c.take<uint32_t>(pad64(m));
    L.rank_r = c.take<uint32_t>(pad64(nr));
    L.id_r = c.take<uint32_t>(pad64(nr));
    return L;
}

struct BuildWs {
    BuildFlags *flags;
    uint32_t *deg_l, *deg_r, *deg_sorted, *ids_in, *ids_out;
    unsigned long long *keys_in, *keys_out;
    uint32_t *vals_in, *vals_out;
    uint32_t *scan_tmp;
    void *sort_tmp;
    size_t sort_tmp_bytes;
};

static size_t sort_tmp_needed(uint32_t nl, uint32_t nr, uint64_t m) {
    size_t a = 0, b = 0;
    uint64_t nmax = nl > nr ? nl : nr;
    const uint64_t big = m > nmax ? m : nmax;
    (void)rocprim::radix_sort_pairs(nullptr, a, (unsigned long long *)nullptr,
                              (unsigned long long *)nullptr, (uint32_t *)nullptr,
                              (uint32_t *)nullptr, (size_t)(big ? big : 1), 0, 64);
    (void)rocprim::radix_sort_pairs(nullptr, b, (uint32_t *)nullptr, (uint32_t *)nullptr,
                              (uint32_t *)nullptr, (uint32_t *)nullptr, (size_t)(nmax ? nmax : 1),
                              0, 32);
    return (a > b ? a : b) + 256;
}

static BuildWs carve_ws(Carver &c, uint32_t nl, uint32_t nr, uint64_t m) {
    BuildWs w;
    uint64_t nmax = nl > nr ? nl : nr;
    w.flags = c.take<BuildFlags>(1);
    w.deg_l = c.take<uint32_t>(pad64(nl));
    w.deg_r = c.take<uint32_t>(pad64(nr));
    w.deg_sorted = c.take<uint32_t>(pad64(nmax));
    w.ids_in = c.take<uint32_t>(pad64(nmax));
    w.ids_out = c.take<uint32_t>(pad64(nmax));
    const uint64_t big = m > nmax ? m : nmax;   // edge keys, or vertex keys of a part-major rank
    w.keys_in = c.take<unsigned long long>(pad64(big));
    w.keys_out = c.take<unsigned long long>(pad64(big));
    w.vals_in = c.take<uint32_t>(pad64(m));
    w.vals_out = c.take<uint32_t>(pad64(m));
    w.scan_tmp = c.take<uint32_t>(scan_tmp_elems(nmax + 1));
    w.sort_tmp_bytes = sort_tmp_needed(nl, nr, m);
    w.sort_tmp = c.take<char>(w.sort_tmp_bytes);
    return w;
}

static int check_sizes(uint32_t nl, uint32_t nr, uint64_t m) {
    const uint64_t lim = 0xFFFFFFFFull - 64;
    if (m >= lim || nl >= lim || nr >= lim) return BFC_E_TOO_LARGE;
    if (m > (uint64_t)nl * (uint64_t)nr) return BFC_E_DUP_EDGE;  // cannot be simple
    return BFC_OK;
}

// Rank one side by (degree, id), or by (part, degree, id) when part offsets
// are given, and build its row offsets.
static int rank_side(uint32_t n, const uint32_t *deg, BuildWs &w, uint32_t *rank, uint32_t *id,
                     uint32_t *off, hipStream_t s, const uint32_t *part = nullptr,
                     uint32_t nparts = 0) {
    if (n == 0) {
        k_fill_u32<<<1, 64, 0, s>>>(off, 1, 0);
        BFC_HIP(hipGetLastError());
        return BFC_OK;
    }
    k_iota<<<grid_for(n), 256, 0, s>>>(w.ids_in, n);
    size_t tb = w.sort_tmp_bytes;
    if (part && nparts > 1) {
        k_part_keys<<<grid_for(n), 256, 0, s>>>(deg, n, part, nparts, w.keys_in);
        BFC_HIP(hipGetLastError());
        const int hb = 32 + bits_for(nparts);
        BFC_HIP(rocprim::radix_sort_pairs(w.sort_tmp, tb, w.keys_in, w.keys_out, w.ids_in, id,
                                          (size_t)n, 0, hb, s));
        k_low_words<<<grid_for(n), 256, 0, s>>>(w.keys_out, n, w.deg_sorted);
    } else {
        BFC_HIP(rocprim::radix_sort_pairs(w.sort_tmp, tb, deg, w.deg_sorted, w.ids_in, id,
                                          (size_t)n, 0, 32, s));
    }
    k_fill_u32<<<1, 64, 0, s>>>(off, 1, 0);
    k_ranks<<<grid_for(n), 256, 0, s>>>(id, w.deg_sorted, n, rank, off + 1);
    BFC_HIP(hipGetLastError());
    return scan_u32_inclusive(off + 1, off + 1, n, w.scan_tmp, s);
}

static int build_csr(const uint32_t *src, const uint32_t *dst, uint64_t m, uint32_t n_dst,
                     const uint32_t *rank_src, const uint32_t *rank_dst, uint32_t n_src,
                     BuildWs &w, uint32_t *adj, uint32_t *eid, hipStream_t s) {
    if (m == 0) return BFC_OK;
    int cb = bits_for(n_dst), rb = bits_for(n_src);
    k_make_keys<<<grid_for(m), 256, 0, s>>>(src, dst, m, rank_src, rank_dst, cb, w.keys_in,
                                             w.vals_in);
    BFC_HIP(hipGetLastError());
    size_t tb = w.sort_tmp_bytes;
    BFC_HIP(rocprim::radix_sort_pairs(w.sort_tmp, tb, w.keys_in, w.keys_out, w.vals_in, eid,
                                      (size_t)m, 0, cb + rb, s));
    uint32_t mask = cb >= 32 ? 0xFFFFFFFFu : ((1u << cb) - 1);
    k_unpack_keys<<<grid_for(m), 256, 0, s>>>(w.keys_out, m, mask, adj, w.flags);
    BFC_HIP(hipGetLastError());
    return BFC_OK;
}

}  // namespace bfc

using namespace bfc;

extern "C" {

const char *bfc_status_str(int code) {
    switch (code) {
        case BFC_OK: return "ok";
        case BFC_E_NULL: return "null pointer";
        case BFC_E_ARG: return "bad argument";
        case BFC_E_ID_RANGE: return "vertex id out of range";
        case BFC_E_DUP_EDGE: return "duplicate edge (graph is not simple)";
        case BFC_E_TOO_LARGE: return "graph too large for 32-bit offsets";
        case BFC_E_WS_SMALL: return "workspace or storage too small";
        case BFC_E_PROBS: return "probabilities negative, NaN, infinite or all zero";
        case BFC_E_OVERFLOW_RISK: return "count could overflow uint64";
        case BFC_E_HIP: return "HIP runtime error";
        case BFC_E_ALIGN: return "device pointer not 256-byte aligned";
        default: return "unknown status";
    }
}

const char *bfc_last_hip_error(void) { return g_hip_err; }

int bfc_graph_storage_size(uint32_t nl, uint32_t nr, uint64_t m, size_t *bytes) {
    if (!bytes) return BFC_E_NULL;
    BFC_TRY(check_sizes(nl, nr, m));
    Carver c(nullptr, 0);
    carve_storage(c, nl, nr, m);
    *bytes = c.used;
    return BFC_OK;
}

int bfc_graph_build_ws_size(uint32_t nl, uint32_t nr, uint64_t m, size_t *bytes) {
    if (!bytes) return BFC_E_NULL;
    BFC_TRY(check_sizes(nl, nr, m));
    Carver c(nullptr, 0);
    carve_ws(c, nl, nr, m);
    *bytes = c.used;
    return BFC_OK;
}

static int build_graph(uint32_t nl, uint32_t nr, uint64_t m, const uint32_t *d_l,
                       const uint32_t *d_r, uint32_t nparts, const uint32_t *part_l,
                       const uint32_t *part_r, void *d_storage, size_t storage_bytes, void *d_ws,
                       size_t ws_bytes, hipStream_t s, bfc_graph *out) {
    if (!out || !d_storage || !d_ws || (m && (!d_l || !d_r))) return BFC_E_NULL;
    BFC_TRY(check_sizes(nl, nr, m));
    if (!aligned256(d_storage) || !aligned256(d_ws)) return BFC_E_ALIGN;
    Carver cs(d_storage, storage_bytes);
    Layout L = carve_storage(cs, nl, nr, m);
    Carver cw(d_ws, ws_bytes);
    BuildWs w = carve_ws(cw, nl, nr, m);
    if (!cs.fits() || !cw.fits()) return BFC_E_WS_SMALL;
    int dev = 0;
    BFC_HIP(hipGetDevice(&dev));

    BFC_HIP(hipMemsetAsync(w.flags, 0, sizeof(BuildFlags), s));
    if (m) {
        k_validate<<<grid_for(m), 256, 0, s>>>(d_l, d_r, m, nl, nr, w.flags);
        BFC_HIP(hipGetLastError());
    }
    BuildFlags hf;
    BFC_HIP(hipMemcpyAsync(&hf, w.flags, sizeof(hf), hipMemcpyDeviceToHost, s));
    BFC_HIP(hipStreamSynchronize(s));
    if (hf.bad_id) return BFC_E_ID_RANGE;

    BFC_HIP(hipMemsetAsync(w.deg_l, 0, sizeof(uint32_t) * pad64(nl), s));
    BFC_HIP(hipMemsetAsync(w.deg_r, 0, sizeof(uint32_t) * pad64(nr), s));
    if (m) {
        k_degrees<<<grid_for(m), 256, 0, s>>>(d_l, d_r, m, w.deg_l, w.deg_r);
        BFC_HIP(hipGetLastError());
    }
    if (nl) {
        k_degree_stats<<<grid_for(nl), 256, 0, s>>>(w.deg_l, nl, &w.flags->sumsq_l, &w.flags->w_l,
                                                     &w.flags->max_deg_l);
    }
    if (nr) {
        k_degree_stats<<<grid_for(nr), 256, 0, s>>>(w.deg_r, nr, &w.flags->sumsq_r, &w.flags->w_r,
                                                     &w.flags->max_deg_r);
    }
    BFC_HIP(hipGetLastError());
    BFC_TRY(rank_side(nl, w.deg_l, w, L.rank_l, L.id_l, L.off_l, s, part_l, nparts));
    BFC_TRY(rank_side(nr, w.deg_r, w, L.rank_r, L.id_r, L.off_r, s, part_r, nparts));
    BFC_TRY(build_csr(d_l, d_r, m, nr, L.rank_l, L.rank_r, nl, w, L.adj_l, L.eid_l, s));
    BFC_TRY(build_csr(d_r, d_l, m, nl, L.rank_r, L.rank_l, nr, w, L.adj_r, L.eid_r, s));
    if (m) {
        // xpos_l[k] = position in adj_r of the edge eid_l[k], and vice versa.
        k_scatter_pos<<<grid_for(m), 256, 0, s>>>(L.eid_r, m, w.vals_in);
        k_gather_pos<<<grid_for(m), 256, 0, s>>>(L.eid_l, m, w.vals_in, L.xpos_l);
        k_scatter_pos<<<grid_for(m), 256, 0, s>>>(L.eid_l, m, w.vals_in);
        k_gather_pos<<<grid_for(m), 256, 0, s>>>(L.eid_r, m, w.vals_in, L.xpos_r);
        BFC_HIP(hipGetLastError());
    }
    BFC_HIP(hipMemcpyAsync(&hf, w.flags, sizeof(hf), hipMemcpyDeviceToHost, s));
    BFC_HIP(hipStreamSynchronize(s));
    if (hf.dup) return BFC_E_DUP_EDGE;

    bfc_graph g;
    memset(&g, 0, sizeof(g));
    g.n_left = nl;
    g.n_right = nr;
    g.n_edges = m;
    g.off_l = L.off_l; g.adj_l = L.adj_l; g.eid_l = L.eid_l; g.xpos_l = L.xpos_l;
    g.rank_l = L.rank_l; g.id_l = L.id_l;
    g.off_r = L.off_r; g.adj_r = L.adj_r; g.eid_r = L.eid_r; g.xpos_r = L.xpos_r;
    g.rank_r = L.rank_r; g.id_r = L.id_r;
    g.sumsq_l = hf.sumsq_l;
    g.sumsq_r = hf.sumsq_r;
    g.wedges_mid_l = hf.w_l;
    g.wedges_mid_r = hf.w_r;
    g.max_deg_l = hf.max_deg_l;
    g.max_deg_r = hf.max_deg_r;
    g.device = dev;
    *out = g;
    return BFC_OK;
}

int bfc_graph_build(uint32_t nl, uint32_t nr, uint64_t m, const uint32_t *d_l,
                    const uint32_t *d_r, void *d_storage, size_t storage_bytes, void *d_ws,
                    size_t ws_bytes, hipStream_t s, bfc_graph *out) {
    return build_graph(nl, nr, m, d_l, d_r, 0, nullptr, nullptr, d_storage, storage_bytes, d_ws,
                       ws_bytes, s, out);
}

int bfc_graph_build_parts(uint32_t nl, uint32_t nr, uint64_t m, const uint32_t *d_l,
                          const uint32_t *d_r, uint32_t nparts, const uint32_t *d_part_l,
                          const uint32_t *d_part_r, void *d_storage, size_t storage_bytes,
                          void *d_ws, size_t ws_bytes, hipStream_t s, bfc_graph *out) {
    if (nparts == 0) return BFC_E_ARG;
    if (!d_part_l || !d_part_r) return BFC_E_NULL;
    return build_graph(nl, nr, m, d_l, d_r, nparts, d_part_l, d_part_r, d_storage, storage_bytes,
                       d_ws, ws_bytes, s, out);
}

}  // extern "C"
