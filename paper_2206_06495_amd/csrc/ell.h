// Device helpers for slot-major ELL operators: entry s of row r is at
// [s * rows + r], so consecutive rows (threads) read consecutive addresses
// for every slot and the index/weight streams are fully coalesced.
#pragma once

#include "common.h"

namespace rbf {

// Sum over the stencil of row `r`: acc += w[s][r] * f(idx[s][r]) for
// each slot.  KT > 0 fixes the stencil width at compile time (all loads of
// the row are issued before the gathers); KT == 0 uses the runtime width k.
// NW weight arrays share one index array (e.g. D_x and D_y of one stencil
// set); the gather functor g(j, v) fills Gather::NV values taken at column j
// (several vectors on one matrix).  FP64 weights and accumulation.
//
// CH (a divisor of KT) bounds register use when the gather returns several
// values: slots are processed CH at a time instead of all KT at once.
// With KT > 0 the index and weight streams use temporal loads: the index
// array of a stencil set is shared by several operators of one time step
// (advection, the viscous right-hand side and sweeps), which then find it
// in the memory-side cache; measured faster than streaming loads for the
// explicit stages at h = 1/400.
template <int KT, int NW, class Gather, int CH = KT>
__device__ __forceinline__ void ell_row(const int *__restrict__ idx, const double *const (&w)[NW],
                                        int64_t rows, int64_t r, int k, Gather g,
                                        double (&acc)[NW][Gather::NV]) {
    if constexpr (KT > 0) {
        static_assert(KT % CH == 0, "chunk must divide the stencil width");
#pragma unroll 1
        for (int s0 = 0; s0 < KT; s0 += CH) {
            int jj[CH];
            double ww[NW][CH];
#pragma unroll
            for (int s = 0; s < CH; ++s) jj[s] = idx[(int64_t)(s0 + s) * rows + r];
#pragma unroll
            for (int s = 0; s < CH; ++s)
#pragma unroll
                for (int o = 0; o < NW; ++o)
                    ww[o][s] = w[o][(int64_t)(s0 + s) * rows + r];
#pragma unroll
            for (int s = 0; s < CH; ++s) {
                double v[Gather::NV];
                g(jj[s], v);
#pragma unroll
                for (int o = 0; o < NW; ++o)
#pragma unroll
                    for (int c = 0; c < Gather::NV; ++c) acc[o][c] = fma(ww[o][s], v[c], acc[o][c]);
            }
        }
    } else {
#pragma unroll 4
        for (int s = 0; s < k; ++s) {
            const int j = ld_stream(idx + (int64_t)s * rows + r);
            double v[Gather::NV];
            g(j, v);
#pragma unroll
            for (int o = 0; o < NW; ++o) {
                const double ws = ld_stream(w[o] + (int64_t)s * rows + r);
#pragma unroll
                for (int c = 0; c < Gather::NV; ++c) acc[o][c] = fma(ws, v[c], acc[o][c]);
            }
        }
    }
}

// Half of row r's stencil for a two-lanes-per-row layout: slots
// half * KT/2 .. (half + 1) * KT/2 - 1 (KT > 0, even); the caller adds the
// two lanes' sums.  Plain (temporal) loads of the operator: its user, the
// viscous Jacobi sweep, reads it once per sweep, several times per solve,
// and it stays in the memory-side cache between sweeps.
template <int KT, class Gather>
__device__ __forceinline__ void ell_half_row(const int *__restrict__ idx,
                                             const double *__restrict__ w, int64_t rows,
                                             int64_t r, int half, Gather g,
                                             double (&acc)[Gather::NV]) {
    static_assert(KT > 0 && KT % 2 == 0, "two halves of a fixed stencil");
    constexpr int H = KT / 2;
    int jj[H];
    double ww[H];
#pragma unroll
    for (int s = 0; s < H; ++s) jj[s] = idx[(int64_t)(half * H + s) * rows + r];
#pragma unroll
    for (int s = 0; s < H; ++s) ww[s] = w[(int64_t)(half * H + s) * rows + r];
#pragma unroll
    for (int s = 0; s < H; ++s) {
        double v[Gather::NV];
        g(jj[s], v);
#pragma unroll
        for (int c = 0; c < Gather::NV; ++c) acc[c] = fma(ww[s], v[c], acc[c]);
    }
}

}  // namespace rbf
