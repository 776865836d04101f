// Shared host/device helpers of the gfx950 RBF-FD library: error state,
// HIP call checking, launch geometry (XCD-aware block remap), reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstdarg>
#include <cstdio>
#include <string>

#include "../../include/rbffd.h"

namespace rbf {

// ---------------------------------------------------------------- errors --
void set_error(const char *fmt, ...);
void clear_error();

#define RBF_HIP(call)                                                            \
    do {                                                                         \
        hipError_t e_ = (call);                                                  \
        if (e_ != hipSuccess) {                                                  \
            ::rbf::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), \
                             __FILE__, __LINE__);                                \
            return (e_ == hipErrorOutOfMemory) ? RBF_E_NOMEM : RBF_E_DEVICE;     \
        }                                                                        \
    } while (0)

#define RBF_ARG(cond, ...)                                                       \
    do {                                                                         \
        if (!(cond)) {                                                           \
            ::rbf::set_error(__VA_ARGS__);                                       \
            return RBF_E_ARG;                                                    \
        }                                                                        \
    } while (0)

#define RBF_CHECK_LAUNCH() RBF_HIP(hipGetLastError())

inline hipStream_t as_stream(rbf_stream s) { return reinterpret_cast<hipStream_t>(s); }

// ------------------------------------------------------------ geometry --
constexpr int kXcds = 8;  // MI355X: 8 accelerator complex dies, 32 CUs each

// Workgroups are dispatched round-robin over the XCDs (block b runs on XCD
// b % 8).  Map them so that each XCD works on one contiguous range of
// logical blocks: rows that share stencil neighbours then share that XCD's
// L2.  The map is a bijection on [0, nblocks).
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t nblocks) {
    uint32_t x = b % kXcds, k = b / kXcds;
    uint32_t q = nblocks / kXcds, r = nblocks % kXcds;
    return (x < r) ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

inline uint32_t blocks_for(int64_t n, int threads) {
    return static_cast<uint32_t>((n + threads - 1) / threads);
}

// Non-temporal (streaming) loads for operator data that is read once per
// application, so that the gathered vectors stay in the caches.
template <class T>
__device__ __forceinline__ T ld_stream(const T *p) {
    return __builtin_nontemporal_load(p);
}

// A double moved across lanes by one DPP control (both 32-bit halves with
// the same pattern; every lane active).
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ double readlane_double(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sums over the two halves of the wave (lanes 0-31 and 32-63), without LDS:
// DPP rotations by 8 and 4 inside each 16-lane row, then quad swaps by 2
// and 1, leave every lane with its row's sum; lanes 0 + 16 and 32 + 48 are
// then read as uniform values.  A fixed order of additions: deterministic.
// Every lane must be active.
__device__ __forceinline__ void half_wave_sums(double v, double &lo, double &hi) {
    v += dpp_move<0x128>(v);  // row_ror:8
    v += dpp_move<0x124>(v);  // row_ror:4
    v += dpp_move<0x4E>(v);   // quad_perm [2,3,0,1]
    v += dpp_move<0xB1>(v);   // quad_perm [1,0,3,2]
    lo = readlane_double(v, 0) + readlane_double(v, 16);
    hi = readlane_double(v, 32) + readlane_double(v, 48);
}

// Wave-level sum of a double (64 lanes): the DPP sums of the four 16-lane
// rows, added as (0 + 16) + (32 + 48); a fixed order of additions, so
// results are deterministic; uniform result.  Every lane must be active.
__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_move<0x128>(v);
    v += dpp_move<0x124>(v);
    v += dpp_move<0x4E>(v);
    v += dpp_move<0xB1>(v);
    return (readlane_double(v, 0) + readlane_double(v, 16)) +
           (readlane_double(v, 32) + readlane_double(v, 48));
}

// Block sum of NV doubles per thread; every thread returns the totals.
// `lds` must hold NV * (blockDim.x / 64) doubles.  Deterministic.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double *lds) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
    __syncthreads();
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i) lds[i * nw + wid] = v[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += lds[i * nw + w];
        v[i] = s;
    }
    __syncthreads();
}

}  // namespace rbf
