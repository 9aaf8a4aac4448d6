// Internal helpers shared by the library's HIP sources (not installed).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "../../include/bfc.h"

namespace bfc {

// ------------------------------------------------------------------ errors
void set_hip_error(hipError_t e);

#define BFC_HIP(call)                                   \
    do {                                                \
        hipError_t e_ = (call);                         \
        if (e_ != hipSuccess) {                         \
            ::bfc::set_hip_error(e_);                   \
            return BFC_E_HIP;                           \
        }                                               \
    } while (0)

#define BFC_TRY(call)                                   \
    do {                                                \
        int rc_ = (call);                               \
        if (rc_ != BFC_OK) return rc_;                  \
    } while (0)

// ------------------------------------------------------------------ workspace carving
// Hands out 256-byte aligned sub-buffers of a caller buffer.  With base ==
// nullptr it only counts bytes (for the *_ws_size queries).
struct Carver {
    char *base;
    size_t cap;
    size_t used = 0;
    Carver(void *b, size_t c) : base((char *)b), cap(c) {}
    template <class T>
    T *take(size_t count) {
        size_t bytes = (count * sizeof(T) + 255) & ~size_t(255);
        if (bytes == 0) bytes = 256;
        T *p = base ? (T *)(base + used) : nullptr;
        used += bytes;
        return p;
    }
    bool fits() const { return base == nullptr || used <= cap; }
};

inline bool aligned256(const void *p) { return ((uintptr_t)p & 255) == 0; }

// Arrays are padded to a multiple of 64 elements so that 16-byte vector
// loads of aligned groups never run past an allocation.
inline size_t pad64(uint64_t n) { return (size_t)((n + 64) & ~uint64_t(63)); }

// Entries readable past the end of an adjacency array: the count kernels load
// whole 16-entry pieces whose tail may run beyond the last list.
constexpr uint64_t ADJ_SLACK = 64;

int device_cu_count(int device);

// ------------------------------------------------------------------ scans
// Inclusive prefix sum of n uint32 values (may alias in/out).  tmp must hold
// scan_tmp_elems(n) uint32.  Sums must fit in uint32.
size_t scan_tmp_elems(uint64_t n);
int scan_u32_inclusive(const uint32_t *in, uint32_t *out, uint64_t n, uint32_t *tmp,
                       hipStream_t s);

// ------------------------------------------------------------------ device helpers
constexpr int WAVE = 64;

// Wave-wide scans on the DPP paths (register to register, no LDS round
// trip): a Hillis-Steele scan inside each row of 16 lanes (row_shr 1, 2, 4,
// 8), then the row totals carried with row_bcast:15 into rows 1 and 3 and
// row_bcast:31 into rows 2 and 3.  Lanes whose DPP source is outside the
// row, or rows the row mask leaves out, read the identity.  Call with all
// 64 lanes active.
template <int CTRL, int ROWS, bool BOUND>
__device__ inline uint32_t dpp_u32(uint32_t ident, uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)ident, (int)v, CTRL, ROWS, 0xf, BOUND);
}

__device__ inline uint32_t wave_incl_scan(uint32_t v) {
    v += dpp_u32<0x111, 0xf, true>(0u, v);
    v += dpp_u32<0x112, 0xf, true>(0u, v);
    v += dpp_u32<0x114, 0xf, true>(0u, v);
    v += dpp_u32<0x118, 0xf, true>(0u, v);
    v += dpp_u32<0x142, 0xa, false>(0u, v);
    v += dpp_u32<0x143, 0xc, false>(0u, v);
    return v;
}

// Inclusive running maximum (identity 0).
__device__ inline uint32_t wave_incl_max(uint32_t v) {
    v = max(v, dpp_u32<0x111, 0xf, true>(0u, v));
    v = max(v, dpp_u32<0x112, 0xf, true>(0u, v));
    v = max(v, dpp_u32<0x114, 0xf, true>(0u, v));
    v = max(v, dpp_u32<0x118, 0xf, true>(0u, v));
    v = max(v, dpp_u32<0x142, 0xa, false>(0u, v));
    v = max(v, dpp_u32<0x143, 0xc, false>(0u, v));
    return v;
}

// Minimum over the wave, returned to every lane (identity 0xFFFFFFFF).
__device__ inline uint32_t wave_min(uint32_t v) {
    const uint32_t I = 0xFFFFFFFFu;
    v = min(v, dpp_u32<0x111, 0xf, false>(I, v));
    v = min(v, dpp_u32<0x112, 0xf, false>(I, v));
    v = min(v, dpp_u32<0x114, 0xf, false>(I, v));
    v = min(v, dpp_u32<0x118, 0xf, false>(I, v));
    v = min(v, dpp_u32<0x142, 0xa, false>(I, v));
    v = min(v, dpp_u32<0x143, 0xc, false>(I, v));
    return (uint32_t)__builtin_amdgcn_readlane((int)v, WAVE - 1);
}

// Value of lane 63 (wave-uniform).
__device__ inline uint32_t wave_last(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, WAVE - 1);
}

__device__ inline unsigned long long wave_sum64(unsigned long long v) {
#pragma unroll
    for (int d = WAVE / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, WAVE);
    return v;
}

// Block-wide exclusive scan of one uint32 per thread (NT threads, NT/64
// waves).  `red` is __shared__ scratch of NT/64 + 1 words.  Returns the
// exclusive prefix; *total receives the block sum.  Contains barriers.
template <int NT>
__device__ inline uint32_t block_excl_scan(uint32_t v, uint32_t *red, uint32_t *total) {
    const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
    uint32_t inc = wave_incl_scan(v);
    if (lane == WAVE - 1) red[wid] = inc;
    __syncthreads();
    uint32_t base = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < NT / WAVE; w++) {
        uint32_t x = red[w];
        if (w < wid) base += x;
        tot += x;
    }
    __syncthreads();
    *total = tot;
    return base + inc - v;
}

template <int NT>
__device__ inline uint32_t block_min(uint32_t v, uint32_t *red) {
    const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
    v = wave_min(v);
    if (lane == 0) red[wid] = v;
    __syncthreads();
    uint32_t m = red[0];
#pragma unroll
    for (int w = 1; w < NT / WAVE; w++) m = min(m, red[w]);
    __syncthreads();
    return m;
}

template <int NT>
__device__ inline unsigned long long block_sum64(unsigned long long v,
                                                 unsigned long long *red) {
    const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
    v = wave_sum64(v);
    if (lane == 0) red[wid] = v;
    __syncthreads();
    unsigned long long s = 0;
#pragma unroll
    for (int w = 0; w < NT / WAVE; w++) s += red[w];
    __syncthreads();
    return s;
}

// First index j in [0, n) with a[j] > x (a non-decreasing), in LDS.
__device__ inline uint32_t upper_bound_lds(const uint32_t *a, uint32_t n, uint32_t x) {
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        if (a[mid] > x) hi = mid; else lo = mid + 1;
    }
    return lo;
}

// First position p in [lo, hi) with a[p] >= x (a ascending), global memory.
__device__ inline uint32_t lower_bound_glb(const uint32_t *a, uint32_t lo, uint32_t hi, uint32_t x) {
    while (lo < hi) {
        uint32_t mid = lo + ((hi - lo) >> 1);
        if (a[mid] < x) lo = mid + 1; else hi = mid;
    }
    return lo;
}

}  // namespace bfc

namespace bfc {
// Local counts of the starts of one side (count.hip); see local_run there.
// split: wedges per part of a wide start (0: the default, 2^24).
int local_ws_size(const bfc_graph *g, int side, size_t *bytes, uint64_t split = 0);
int local_run(const bfc_graph *g, int side, const uint8_t *mark_rank, uint64_t *d_cnt_l,
              uint64_t *d_cnt_r, uint64_t *d_cnt_e, void *d_ws, size_t ws_bytes, hipStream_t s,
              uint64_t split = 0);
// Workspace bfc_exact needs on any graph of these sizes.
size_t exact_ws_bound(uint32_t nl, uint32_t nr, uint64_t m);
}  // namespace bfc
