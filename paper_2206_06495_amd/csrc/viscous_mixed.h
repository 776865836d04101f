// Mixed-precision viscous solve (eq. (16)): FP32 Jacobi sweeps inside FP64
// iterative refinement.  Included by solver.hip inside its anonymous
// namespace.
//
// Both velocity components are solved together with H = I - a D_Lap (the
// Crank-Nicolson matrix, identity rows on walls).  Outer iteration i:
//   r_i = b - H x_i                     FP64 operator, FP64 vectors
//   (test ||r_i|| <= tol ||b|| per component: x_i is accepted)
//   d_0 = D^-1 r_i,  d_{s+1} = d_s + D^-1 (r_i - H d_s)  (s < kHMixSweeps)
//                                       FP32 weights, vectors and sums
//   x_{i+1} = x_i + d                   FP64
// The outer residual and the iterate stay FP64, so the accepted x solves the
// FP64 system to the requested tolerance; the FP32 sweeps only supply the
// corrections.  They run when H's Jacobi bound (max_i sum_{j != i}
// |h_ij| / |h_ii|) is at most kJacobiMax, so each sweep contracts the
// correction's error by that factor or better.
#pragma once

constexpr int kHMixSweeps = 2;  // FP32 sweeps per outer iteration (after d_0)

struct HMix {
    const int *idx;
    const float *w32;     // [k][N] FP32 copy of H
    const float *dinv32;  // [N] FP32 1 / h_ii
    int64_t n;
    int k;
    double2 *x;           // [N] FP64 iterate, components interleaved
    float2 *r;            // [N] FP32 residual of the current outer iteration
    float2 *d[2];         // [N] FP32 corrections, by sweep parity
    double *part;         // [2 parities][4][kMaxBlocks]: ||r_c||^2, ||b_c||^2
    int *flag;            // flag (0 running, 1 accepted, -1 non-finite), accepted index
};

__global__ void k_hm_clear(int *flag) {
    if (threadIdx.x < 2) flag[threadIdx.x] = 0;
}

// Outer residual r_i = b - H x_i and d_0 = D^-1 r_i, with block partials of
// ||r_i||^2 and ||b||^2 per component (slot i & 1).  FIRST: x_0 comes from
// the caller's [2][N] guess and is stored interleaved.
template <int KT, bool FIRST>
__global__ void __launch_bounds__(kThreads) k_hm_res(EllM A, const double *__restrict__ b,
                                                      const double *__restrict__ x0, HMix X, int i) {
    if (X.flag[0] != 0) return;
    double acc[2 * kHR] = {};
    for (int64_t it = 0;; ++it) {
        const int64_t row = row_of(it);
        if (row - threadIdx.x >= A.n) break;
        if (row < A.n) {
            double ax[1][kHR] = {};
            const double *ws[1] = {A.w};
            double xs[kHR];
            if constexpr (FIRST) {
                rbf::ell_row<KT, 1>(A.idx, ws, A.n, row, A.k, GatherN<kHR>{x0, A.n}, ax);
                xs[0] = x0[row];
                xs[1] = x0[A.n + row];
                X.x[row] = make_double2(xs[0], xs[1]);
            } else {
                rbf::ell_row<KT, 1>(A.idx, ws, A.n, row, A.k, GatherI2{X.x}, ax);
            }
            const float di = X.dinv32[row];
            float rr[kHR];
#pragma unroll
            for (int c = 0; c < kHR; ++c) {
                const double bv = b[c * A.n + row], rv = bv - ax[0][c];
                rr[c] = (float)rv;
                acc[c] += rv * rv;
                acc[kHR + c] += bv * bv;
            }
            X.r[row] = make_float2(rr[0], rr[1]);
            X.d[0][row] = make_float2(di * rr[0], di * rr[1]);
        }
    }
    __shared__ double lds[2 * kHR * (kThreads / 64)];
    rbf::block_sum<2 * kHR>(acc, lds);
    if (threadIdx.x == 0) {
        double *pp = X.part + (int64_t)(i & 1) * 2 * kHR * kMaxBlocks;
#pragma unroll
        for (int c = 0; c < 2 * kHR; ++c) pp[(int64_t)c * kMaxBlocks + blockIdx.x] = acc[c];
    }
}

// One FP32 sweep d_{s+1} = d_s + D^-1 (r - H d_s) (s = sweep index, d_s in
// X.d[s & 1]).  TEST (first sweep of an outer iteration): every block first
// reduces the outer residual's partials (same order in every block) and
// all stop when x_i passes, or when a partial is not finite.  LAST: the
// correction is added to the FP64 iterate instead of being stored.
template <int KT, bool TEST, bool LAST>
__global__ void __launch_bounds__(kThreads) k_hm_sweep(HMix X, int i, int s, double tol2, int nbres) {
    if constexpr (TEST) {
        double q[2 * kHR] = {};
        const double *pp = X.part + (int64_t)(i & 1) * 2 * kHR * kMaxBlocks;
        for (int bk = threadIdx.x; bk < nbres; bk += blockDim.x)
#pragma unroll
            for (int c = 0; c < 2 * kHR; ++c) q[c] += pp[(int64_t)c * kMaxBlocks + bk];
        if (X.flag[0] != 0) return;
        __shared__ double lds[2 * kHR * (kThreads / 64)];
        rbf::block_sum<2 * kHR>(q, lds);
        bool conv = true, bad = false;
#pragma unroll
        for (int c = 0; c < kHR; ++c) {
            bad = bad || !isfinite(q[c]) || !isfinite(q[kHR + c]);
            conv = conv && (q[c] <= tol2 * fmax(q[kHR + c], 1e-300) || q[c] == 0.0);
        }
        if (bad || conv) {
            if (blockIdx.x == 0 && threadIdx.x == 0) {
                X.flag[1] = i;
                X.flag[0] = bad ? -1 : 1;
            }
            return;
        }
    } else {
        if (X.flag[0] != 0) return;
    }
    const float2 *din = X.d[s & 1];
    float2 *dout = X.d[(s & 1) ^ 1];
    for (int64_t it = 0;; ++it) {
        const int64_t row = row_of(it);
        if (row - threadIdx.x >= X.n) break;
        if (row < X.n) {
            float a0 = 0.0f, a1 = 0.0f;
            if constexpr (KT > 0) {
                int jj[KT];
                float ww[KT];
                // Temporal loads: every sweep of the solve reads the operator
                // again, and it stays in the memory-side cache between them.
#pragma unroll
                for (int q = 0; q < KT; ++q) jj[q] = X.idx[(int64_t)q * X.n + row];
#pragma unroll
                for (int q = 0; q < KT; ++q) ww[q] = X.w32[(int64_t)q * X.n + row];
#pragma unroll
                for (int q = 0; q < KT; ++q) {
                    const float2 t = din[jj[q]];
                    a0 = fmaf(ww[q], t.x, a0);
                    a1 = fmaf(ww[q], t.y, a1);
                }
            } else {
                for (int q = 0; q < X.k; ++q) {
                    const float wq = X.w32[(int64_t)q * X.n + row];
                    const float2 t = din[X.idx[(int64_t)q * X.n + row]];
                    a0 = fmaf(wq, t.x, a0);
                    a1 = fmaf(wq, t.y, a1);
                }
            }
            const float di = X.dinv32[row];
            const float2 rv = X.r[row], dv = din[row];
            const float n0 = dv.x + di * (rv.x - a0), n1 = dv.y + di * (rv.y - a1);
            if constexpr (LAST) {
                const double2 xv = X.x[row];
                X.x[row] = make_double2(xv.x + (double)n0, xv.y + (double)n1);
            } else {
                dout[row] = make_float2(n0, n1);
            }
        }
    }
}
