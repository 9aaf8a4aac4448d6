// Disjoint unions of many bipartite graphs for batched counting.
//
// A batch of graphs is counted as one graph: the disjoint union of its
// parts, each part entered with the side it should start from (ExactBFC's
// side choice of Sec. 4, made per part) as the union's L.  Butterflies never
// span two parts, so the union's count split by part is each graph's count,
// and one plan plus one persistent launch per kernel class serves the whole
// batch (bfc_exact_parts).
#include "common.h"

#include <vector>

namespace bfc {

// Part of edge e: the last q with eoff[q] <= e (eoff ascending, ng + 1 entries).
__device__ inline uint32_t part_of(const uint64_t *eoff, uint32_t ng, uint64_t e) {
    uint32_t lo = 0, hi = ng;               // answer in [lo, hi)
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (eoff[mid] <= e) lo = mid; else hi = mid;
    }
    return lo;
}

struct UnionArgs {
    const uint64_t *eoff;       // ng + 1
    const uint64_t *loff, *roff; // ng + 1: first slot of each part in degL / degR
    uint32_t ng;
    uint64_t m;
    const uint32_t *l, *r;
};

__global__ void k_union_degrees(UnionArgs a, uint32_t *degL, uint32_t *degR, uint32_t *bad) {
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < a.m;
         e += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t q = part_of(a.eoff, a.ng, e);
        const uint64_t nl = a.loff[q + 1] - a.loff[q], nr = a.roff[q + 1] - a.roff[q];
        const uint32_t l = a.l[e], r = a.r[e];
        if (l >= nl || r >= nr) {
            atomicOr(bad, 1u);
            continue;
        }
        atomicAdd(&degL[a.loff[q] + l], 1u);
        atomicAdd(&degR[a.roff[q] + r], 1u);
    }
}

// sums[2q] = sum of squared L degrees of part q, sums[2q + 1] of R degrees.
__global__ __launch_bounds__(256) void k_union_sumsq(const uint64_t *loff, const uint64_t *roff,
                                                     uint32_t ng, const uint32_t *degL,
                                                     const uint32_t *degR,
                                                     unsigned long long *sums) {
    __shared__ unsigned long long red[256 / WAVE];
    for (uint32_t q = blockIdx.x; q < ng; q += gridDim.x) {
        unsigned long long sl = 0, sr = 0;
        for (uint64_t i = loff[q] + threadIdx.x; i < loff[q + 1]; i += blockDim.x)
            sl += (unsigned long long)degL[i] * degL[i];
        for (uint64_t i = roff[q] + threadIdx.x; i < roff[q + 1]; i += blockDim.x)
            sr += (unsigned long long)degR[i] * degR[i];
        sl = block_sum64<256>(sl, red);
        sr = block_sum64<256>(sr, red);
        if (threadIdx.x == 0) {
            sums[2 * q] = sl;
            sums[2 * q + 1] = sr;
        }
    }
}

// Union ids; may run in place (ul == l, ur == r): each edge is read before
// it is written, by the same thread.
__global__ void k_union_ids(UnionArgs a, const uint32_t *uoffL, const uint32_t *uoffR,
                            const uint8_t *swapped, uint32_t *ul, uint32_t *ur) {
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < a.m;
         e += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t q = part_of(a.eoff, a.ng, e);
        const uint32_t l = a.l[e], r = a.r[e];
        const bool sw = swapped[q] != 0;
        ul[e] = uoffL[q] + (sw ? r : l);
        ur[e] = uoffR[q] + (sw ? l : r);
    }
}

static inline unsigned grid_for(uint64_t n, int nt = 256) {
    uint64_t g = (n + nt - 1) / nt;
    if (g < 1) g = 1;
    if (g > 65535ull * 16) g = 65535ull * 16;
    return (unsigned)g;
}

struct UnionWs {
    uint64_t *eoff, *loff, *roff;
    uint32_t *degL, *degR, *bad, *uoffL, *uoffR;
    uint8_t *swapped;
    unsigned long long *sums;
};

static void carve_union(Carver &c, uint32_t ng, uint64_t sum_l, uint64_t sum_r, UnionWs &w) {
    w.eoff = c.take<uint64_t>(ng + 1);
    w.loff = c.take<uint64_t>(ng + 1);
    w.roff = c.take<uint64_t>(ng + 1);
    w.degL = c.take<uint32_t>(pad64(sum_l));
    w.degR = c.take<uint32_t>(pad64(sum_r));
    w.bad = c.take<uint32_t>(1);
    w.uoffL = c.take<uint32_t>(ng + 1);
    w.uoffR = c.take<uint32_t>(ng + 1);
    w.swapped = c.take<uint8_t>(ng + 1);
    w.sums = c.take<unsigned long long>(2 * (uint64_t)ng);
}

static int union_sizes(uint32_t ng, const uint32_t *h_nl, const uint32_t *h_nr,
                       const uint64_t *h_eoff, uint64_t &sum_l, uint64_t &sum_r) {
    if (!h_nl || !h_nr || !h_eoff) return BFC_E_NULL;
    if (ng == 0) return BFC_E_ARG;
    sum_l = sum_r = 0;
    for (uint32_t q = 0; q < ng; q++) {
        if (h_eoff[q + 1] < h_eoff[q]) return BFC_E_ARG;
        sum_l += h_nl[q];
        sum_r += h_nr[q];
    }
    if (h_eoff[0] != 0) return BFC_E_ARG;
    return BFC_OK;
}

}  // namespace bfc

using namespace bfc;

extern "C" {

int bfc_batch_union_ws_size(uint32_t ng, const uint32_t *h_nl, const uint32_t *h_nr,
                            const uint64_t *h_eoff, size_t *bytes) {
    if (!bytes) return BFC_E_NULL;
    uint64_t sl, sr;
    BFC_TRY(union_sizes(ng, h_nl, h_nr, h_eoff, sl, sr));
    Carver c(nullptr, 0);
    UnionWs w;
    carve_union(c, ng, sl, sr, w);
    *bytes = c.used;
    return BFC_OK;
}

int bfc_batch_union(uint32_t ng, const uint32_t *h_nl, const uint32_t *h_nr,
                    const uint64_t *h_eoff, const uint32_t *d_l, const uint32_t *d_r,
                    uint32_t *d_ul, uint32_t *d_ur, uint32_t *h_part_l, uint32_t *h_part_r,
                    uint8_t *h_swapped, void *d_ws, size_t ws_bytes, hipStream_t s) {
    if (!h_part_l || !h_part_r || !h_swapped || !d_ws) return BFC_E_NULL;
    uint64_t sl, sr;
    BFC_TRY(union_sizes(ng, h_nl, h_nr, h_eoff, sl, sr));
    const uint64_t m = h_eoff[ng];
    if (m && (!d_l || !d_r || !d_ul || !d_ur)) return BFC_E_NULL;
    if (!aligned256(d_ws)) return BFC_E_ALIGN;
    Carver c(d_ws, ws_bytes);
    UnionWs w;
    carve_union(c, ng, sl, sr, w);
    if (!c.fits()) return BFC_E_WS_SMALL;

    std::vector<uint64_t> loff(ng + 1), roff(ng + 1);
    loff[0] = roff[0] = 0;
    for (uint32_t q = 0; q < ng; q++) {
        loff[q + 1] = loff[q] + h_nl[q];
        roff[q + 1] = roff[q] + h_nr[q];
    }
    BFC_HIP(hipMemcpyAsync(w.eoff, h_eoff, (ng + 1) * sizeof(uint64_t), hipMemcpyHostToDevice, s));
    BFC_HIP(hipMemcpyAsync(w.loff, loff.data(), (ng + 1) * sizeof(uint64_t),
                           hipMemcpyHostToDevice, s));
    BFC_HIP(hipMemcpyAsync(w.roff, roff.data(), (ng + 1) * sizeof(uint64_t),
                           hipMemcpyHostToDevice, s));
    BFC_HIP(hipMemsetAsync(w.degL, 0, pad64(sl) * 4, s));
    BFC_HIP(hipMemsetAsync(w.degR, 0, pad64(sr) * 4, s));
    BFC_HIP(hipMemsetAsync(w.bad, 0, 4, s));
    UnionArgs a = {w.eoff, w.loff, w.roff, ng, m, d_l, d_r};
    unsigned ge = grid_for(m);
    if (ge > 16384) ge = 16384;
    if (m) k_union_degrees<<<ge, 256, 0, s>>>(a, w.degL, w.degR, w.bad);
    k_union_sumsq<<<ng < 65535u ? ng : 65535u, 256, 0, s>>>(w.loff, w.roff, ng, w.degL, w.degR,
                                                            w.sums);
    BFC_HIP(hipGetLastError());
    std::vector<unsigned long long> sums(2 * (size_t)ng);
    uint32_t bad = 0;
    BFC_HIP(hipMemcpyAsync(sums.data(), w.sums, sums.size() * 8, hipMemcpyDeviceToHost, s));
    BFC_HIP(hipMemcpyAsync(&bad, w.bad, 4, hipMemcpyDeviceToHost, s));
    BFC_HIP(hipStreamSynchronize(s));
    if (bad) return BFC_E_ID_RANGE;

    // ExactBFC's rule per part: start from R iff sum_L d^2 < sum_R d^2.
    std::vector<uint32_t> uoffL(ng + 1), uoffR(ng + 1);
    uint64_t ul = 0, ur = 0;
    for (uint32_t q = 0; q < ng; q++) {
        h_swapped[q] = sums[2 * q] < sums[2 * q + 1] ? 1 : 0;
        if (ul > 0xFFFFFFFFull || ur > 0xFFFFFFFFull) return BFC_E_TOO_LARGE;
        h_part_l[q] = uoffL[q] = (uint32_t)ul;
        h_part_r[q] = uoffR[q] = (uint32_t)ur;
        ul += h_swapped[q] ? h_nr[q] : h_nl[q];
        ur += h_swapped[q] ? h_nl[q] : h_nr[q];
    }
    if (ul > 0xFFFFFFFFull || ur > 0xFFFFFFFFull) return BFC_E_TOO_LARGE;
    h_part_l[ng] = uoffL[ng] = (uint32_t)ul;
    h_part_r[ng] = uoffR[ng] = (uint32_t)ur;
    BFC_HIP(hipMemcpyAsync(w.uoffL, uoffL.data(), (ng + 1) * 4, hipMemcpyHostToDevice, s));
    BFC_HIP(hipMemcpyAsync(w.uoffR, uoffR.data(), (ng + 1) * 4, hipMemcpyHostToDevice, s));
    BFC_HIP(hipMemcpyAsync(w.swapped, h_swapped, ng, hipMemcpyHostToDevice, s));
    if (m) k_union_ids<<<ge, 256, 0, s>>>(a, w.uoffL, w.uoffR, w.swapped, d_ul, d_ur);
    BFC_HIP(hipGetLastError());
    BFC_HIP(hipStreamSynchronize(s));
    return BFC_OK;
}

}  // extern "C"
