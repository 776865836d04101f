// Dense FP64 products on the CDNA matrix cores for the n x n transforms of
// the lattice preconditioner (n = K - 1, a few hundred): C = A op(B) with
//   A(i, k)     at A[i + k n]   (column-major),
//   op(B)(k, j) at B[j + k n]   (B row-major, or B^T column-major),
// so that both operands are read with unit stride across the lanes that
// hold consecutive i (A) or j (op(B)).
//
// v_mfma_f64_16x16x4f64, per step k0: lane l supplies A(l%16, k0 + l/16)
// and op(B)(k0 + l/16, l%16); register r of lane l accumulates
// D(4 r + l/16, l%16).
//
// A workgroup of S waves computes one 16x16 tile; wave w takes a contiguous
// share of the k steps (split-K, so the dependent MFMA chain per wave is
// short), loads its operands a chunk ahead of the MFMAs that use them, and
// the S partial tiles are summed through LDS by wave 0.  Ragged edges are
// zero-filled.  The epilogue functor receives (i, j, value) for every
// in-range element of the tile, on wave 0; the return value tells the
// calling wave whether it holds the tile (wave 0) or not.  Every wave of
// the workgroup must call it (it synchronises the workgroup when S > 1).
#pragma once

#include <hip/hip_runtime.h>

namespace rbf {

typedef double dgemm_acc4 __attribute__((ext_vector_type(4)));

template <int S, class Epi>
__device__ __forceinline__ bool dgemm_tile_16x16(int n, const double *__restrict__ A,
                                                 const double *__restrict__ B, int ti, int tj,
                                                 Epi epi) {
    constexpr int C = 8;  // k steps per chunk
    __shared__ dgemm_acc4 red[S > 1 ? S - 1 : 1][64];
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int lr = l & 15, lk = l >> 4;
    const int ia = ti * 16 + lr, jb = tj * 16 + lr;
    const bool in_i = ia < n, in_j = jb < n;
    const int steps = (n + 3) >> 2;
    const int per = (steps + S - 1) / S;
    const int s0 = w * per, s1 = min(steps, s0 + per);
    auto load = [&](int sb, double (&a)[C], double (&b)[C]) {
#pragma unroll
        for (int g = 0; g < C; ++g) {
            const int k = 4 * (sb + g) + lk;
            const bool ok = (sb + g < s1) && k < n;
            a[g] = (ok && in_i) ? A[ia + (int64_t)k * n] : 0.0;
            b[g] = (ok && in_j) ? B[jb + (int64_t)k * n] : 0.0;
        }
    };
    dgemm_acc4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
    double a[C], b[C];
    load(s0, a, b);
    for (int sb = s0; sb < s1; sb += C) {
        double an[C], bn[C];
        if (sb + C < s1) load(sb + C, an, bn);
#pragma unroll
        for (int g = 0; g < C; g += 2) {
            if (sb + g < s1) acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[g], b[g], acc0, 0, 0, 0);
            if (sb + g + 1 < s1)
                acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[g + 1], b[g + 1], acc1, 0, 0, 0);
        }
#pragma unroll
        for (int g = 0; g < C; ++g) {
            a[g] = an[g];
            b[g] = bn[g];
        }
    }
    acc0 += acc1;
    if constexpr (S > 1) {
        if (w > 0) red[w - 1][l] = acc0;
        __syncthreads();
        if (w != 0) return false;
#pragma unroll
        for (int v = 0; v < S - 1; ++v) acc0 += red[v][l];
    }
    const int j = tj * 16 + lr;
    if (j < n) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = ti * 16 + 4 * r + lk;
            if (i < n) epi(i, j, acc0[r]);
        }
    }
    return true;
}

}  // namespace rbf
