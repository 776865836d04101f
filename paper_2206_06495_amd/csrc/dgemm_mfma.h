// Dense products on the CDNA matrix cores for the n x n transforms of the
// lattice preconditioner (n = K - 1, a few hundred), in FP64
// (v_mfma_f64_16x16x4f64) or FP32 (v_mfma_f32_16x16x4f32):
//   C = A op(B),  A(i, k) at A[i + k n] (column-major),
//                 op(B)(k, j) at B[j + k n] (B row-major, or B^T column-major),
// so that both operands are read with unit stride across the lanes that
// hold consecutive i (A) or j (op(B)).
//
// Per MFMA step k0, lane l supplies A(l%16, k0 + l/16) and
// op(B)(k0 + l/16, l%16).  Register r of lane l accumulates D(i, l%16) with
// i = 4 r + l/16 for FP64 and i = 4 (l/16) + r for FP32 (the two
// instructions lay out their 16x16 results differently).
//
// A workgroup of TM * TN * S waves computes a (16 TM) x (16 TN) block: wave
// w owns the 16x16 sub-tile (w % TM, (w / TM) % TN) and the k-share
// w / (TM TN) (split-K, so the dependent MFMA chain per wave is short).
// The waves of one sub-tile read the same operand rows as their neighbours
// in the block, which the CU's L1 serves.  Operands are loaded C k-steps
// at a time, one chunk ahead of the MFMAs that use them (ONESHOT: the
// caller guarantees that a wave's share is at most C steps, and all of it
// is loaded before the first MFMA); the S partial tiles are summed through
// LDS.  Ragged edges are zero-filled.  The epilogue functor receives
// (i, j, value) for every in-range element, on the waves with k-share 0;
// the return value tells the calling wave whether it holds a result.
// Every wave of the workgroup must call it (it synchronises when S > 1).
#pragma once

#include <hip/hip_runtime.h>

namespace rbf {

template <class T>
struct mfma16;
template <>
struct mfma16<double> {
    typedef double acc4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ acc4 step(double a, double b, acc4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int r, int lk) { return 4 * r + lk; }
};
template <>
struct mfma16<float> {
    typedef float acc4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ acc4 step(float a, float b, acc4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int r, int lk) { return 4 * lk + r; }
};

template <class T, int TM, int TN, int S, int C, bool ONESHOT, class Epi>
__device__ __forceinline__ bool mfma_block(int n, const T *__restrict__ A, const T *__restrict__ B,
                                           int bm, int bn, Epi epi) {
    using M = mfma16<T>;
    using acc4 = typename M::acc4;
    constexpr int NT = TM * TN;
    __shared__ acc4 red[S > 1 ? S - 1 : 1][NT][64];
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int wt = w % NT, ws = w / NT;
    const int ti = bm * TM + wt % TM, tj = bn * TN + wt / TM;
    const int lr = l & 15, lk = l >> 4;
    const int ia = ti * 16 + lr, jb = tj * 16 + lr;
    const bool in_i = ia < n, in_j = jb < n;
    const int steps = (n + 3) >> 2;
    const int per = (steps + S - 1) / S;
    const int s0 = ws * per, s1 = min(steps, s0 + per);
    auto load = [&](int sb, T (&a)[C], T (&b)[C]) {
#pragma unroll
        for (int g = 0; g < C; ++g) {
            const int k = 4 * (sb + g) + lk;
            const bool ok = (sb + g < s1) && k < n;
            a[g] = (ok && in_i) ? A[ia + (int64_t)k * n] : T(0);
            b[g] = (ok && in_j) ? B[jb + (int64_t)k * n] : T(0);
        }
    };
    acc4 acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
    T a[C], b[C];
    load(s0, a, b);
    if constexpr (ONESHOT) {
        // The whole k-share fits in one chunk (per <= C, checked by the
        // caller): every operand load is in flight before the first MFMA.
#pragma unroll
        for (int g = 0; g < C; g += 2) {
            if (s0 + g < s1) acc0 = M::step(a[g], b[g], acc0);
            if (g + 1 < C && s0 + g + 1 < s1) acc1 = M::step(a[g + 1], b[g + 1], acc1);
        }
    } else for (int sb = s0; sb < s1; sb += C) {
        T an[C], bn_[C];
        if (sb + C < s1) load(sb + C, an, bn_);
#pragma unroll
        for (int g = 0; g < C; g += 2) {
            if (sb + g < s1) acc0 = M::step(a[g], b[g], acc0);
            if (sb + g + 1 < s1) acc1 = M::step(a[g + 1], b[g + 1], acc1);
        }
#pragma unroll
        for (int g = 0; g < C; ++g) {
            a[g] = an[g];
            b[g] = bn_[g];
        }
    }
    acc0 += acc1;
    if constexpr (S > 1) {
        if (ws > 0) red[ws - 1][wt][l] = acc0;
        __syncthreads();
        if (ws != 0) return false;
#pragma unroll
        for (int v = 0; v < S - 1; ++v) acc0 += red[v][wt][l];
    }
    const int j = tj * 16 + lr;
    if (j < n) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = ti * 16 + M::row(r, lk);
            if (i < n) epi(i, j, acc0[r]);
        }
    }
    return true;
}

}  // namespace rbf
