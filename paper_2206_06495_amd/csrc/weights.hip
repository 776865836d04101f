// rbf_assemble_weights: batched local PHS+poly RBF-FD weight solves.
//
// Sec. 2.1 (eqs. (3)-(9)): for evaluation node x_0 with stencil x_1..x_n,
//   [A P; P^T 0] [w; c] = [L phi; L P],  A_ij = ||x_i - x_j||^m,
// P_jt = the monomials of degree <= q at x_j, right-hand sides L applied to
// phi(||x - x_j||) and to the monomials at x = x_0; w is kept.
//
// One wavefront (64 lanes) solves one system.  Lane i owns row i of the
// augmented matrix (s = n + K_p <= 64 rows) in registers; LU with partial
// pivoting runs across lanes: the pivot is found by a butterfly arg-max over
// the wave, its row is broadcast with v_readlane (scalar operands of the
// updates), and every other unfinished row eliminates with it (row swaps are
// virtual: each lane remembers the step at which its row became pivot).
// The residual of the refinement step recomputes the lane's row of the
// original matrix instead of keeping a copy in registers.  All right-hand sides (one per operator) are
// eliminated together.  One step of iterative refinement with a residual
// accumulated in double-FP64 arithmetic (exact products via fma) brings the
// solution to within a few ulps of the exact solution of the FP64 system.
//
// Local coordinates: x~ = (x_j - x_0) * 2^-e with e = ceil(E/2),
// max_j |x_j - x_0|^2 = f 2^E, 1/2 <= f < 1 (exact scaling); weights are
// returned as w~ * 2^(-e * order).  Matrix and right-hand-side entries are
// computed with separately rounded operations (file built with
// -ffp-contract=off): squared distances dx*dx + dy*dy, r = sqrt(d^2),
// r^m = (d^2)^((m-1)/2) * r as a left-to-right product chain.
// A system is reported singular when a pivot is not larger than
// 16 eps max|A_aug| (e.g. duplicated stencil nodes) or a weight is not finite.
//
// Optional 1-norm condition estimate of the local system (Sec. 4 studies the
// conditioning of these matrices): ||A_aug||_1 exactly (A_aug is symmetric,
// so its largest absolute column sum is its largest absolute row sum) times a
// lower estimate of ||A_aug^-1||_1 from Hager's method with Higham's
// safeguards (Hager 1984; Higham 1988, ACM TOMS 14, the algorithm of
// LAPACK's xLACON): at most five power-like steps x -> sign(A^-1 x) ->
// A^-T sign(..) -> unit vector at the largest entry, then the alternating
// test vector.  A^-T = A^-1 here, so every step is one solve with the LU
// factors.
#include <climits>

#include "common.h"

namespace {

constexpr int kMaxOps = 4;

struct OpSet {
    int n;               // number of operators
    int code[kMaxOps];   // RBF_OP_* codes
    int order[kMaxOps];  // derivative order (scaling exponent multiplier)
};

__device__ __forceinline__ double readlane_d(double v, int l) {
    long long b = __double_as_longlong(v);
    int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
    int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Cross-lane reductions without LDS traffic: DPP moves inside each 16-lane
// row (rotations by 8 and 4, then quad swaps of 2 and 1 leave every lane of
// a row with the row's result), then the four rows' results read by
// v_readlane and combined uniformly.  Exact maxima, so the reduction order
// does not matter; ties of the arg-max go to the lowest lane.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <int CTRL>
__device__ __forceinline__ void dpp_argmax_step(double &c, int &cl) {
    const double ov = dpp_d<CTRL>(c);
    const int ol = __builtin_amdgcn_update_dpp(0, cl, CTRL, 0xF, 0xF, false);
    const bool take = ov > c || (ov == c && ol < cl);
    c = take ? ov : c;
    cl = take ? ol : cl;
}

constexpr int kDppRor8 = 0x128, kDppRor4 = 0x124, kDppSwap2 = 0x4E, kDppSwap1 = 0xB1;

// Lane of the largest c over the wave (lowest lane on ties), wave-uniform.
__device__ __forceinline__ int wave_argmax(double c, int lane) {
    int cl = lane;
    dpp_argmax_step<kDppRor8>(c, cl);
    dpp_argmax_step<kDppRor4>(c, cl);
    dpp_argmax_step<kDppSwap2>(c, cl);
    dpp_argmax_step<kDppSwap1>(c, cl);
    double bv = readlane_d(c, 0);
    int bl = __builtin_amdgcn_readlane(cl, 0);
#pragma unroll
    for (int r = 16; r < 64; r += 16) {
        const double v = readlane_d(c, r);
        const int l = __builtin_amdgcn_readlane(cl, r);
        const bool take = v > bv || (v == bv && l < bl);
        bv = take ? v : bv;
        bl = take ? l : bl;
    }
    return __builtin_amdgcn_readfirstlane(bl);
}

// Largest v over the wave (fmax: NaN only if every lane is NaN), uniform.
__device__ __forceinline__ double wave_max(double v) {
    v = fmax(v, dpp_d<kDppRor8>(v));
    v = fmax(v, dpp_d<kDppRor4>(v));
    v = fmax(v, dpp_d<kDppSwap2>(v));
    v = fmax(v, dpp_d<kDppSwap1>(v));
    return fmax(fmax(readlane_d(v, 0), readlane_d(v, 16)), fmax(readlane_d(v, 32), readlane_d(v, 48)));
}

__device__ __forceinline__ double ipow(double b, int n) {
    if (n == 0) return 1.0;
    double t = b;
    for (int i = 1; i < n; ++i) t = t * b;
    return t;
}

// t^a (0 <= a <= 5) as the product chain ((t t) t)..., without a table
// (a table indexed by a runtime exponent would live in scratch memory).
__device__ __forceinline__ double pow_chain(double t, int a) {
    double r = 1.0, p = t;
#pragma unroll
    for (int i = 1; i <= 5; ++i) {
        r = (i == a) ? p : r;
        p = p * t;
    }
    return r;
}

// Graded monomial index t -> exponents (a, b): degree d, b = t - d(d+1)/2.
__device__ __forceinline__ void mono_exp(int t, int &a, int &b) {
    int d = 0;
    while ((d + 1) * (d + 2) / 2 <= t) ++d;
    b = t - d * (d + 1) / 2;
    a = d - b;
}

// Wave-uniform sum of v over the 64 lanes (lane 0's butterfly result).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return readlane_d(v, 0);
}

// Lane index of the largest |v| among lanes < s (lowest lane on ties),
// wave-uniform.
__device__ __forceinline__ int wave_argmax_abs(double v, int lane, int s) {
    double c = (lane < s) ? fabs(v) : -1.0;
    int cl = lane;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const double ov = __shfl_xor(c, off, 64);
        const int ol = __shfl_xor(cl, off, 64);
        const bool take = ov > c || (ov == c && ol < cl);
        c = take ? ov : c;
        cl = take ? ol : cl;
    }
    return __builtin_amdgcn_readfirstlane(cl);
}

// Solve A x = r with the factors of k_weights' LU: lane i holds r_i and
// receives x_i (0 beyond s).  a holds the multipliers of the steps that
// eliminated this lane's row and its row of U; pl[kk] is the lane that
// pivoted at step kk.
template <int SMAX>
__device__ __forceinline__ double lu_solve_lane(double r, const double (&a)[SMAX], int mystep,
                                                double myinv, const int *pl, int s, int lane) {
#pragma unroll
    for (int kk = 0; kk < SMAX; ++kk) {
        if (kk < s) {
            const double yk = readlane_d(r, pl[kk]);
            if (mystep > kk && mystep != INT_MAX) r = fma(-a[kk], yk, r);
        }
    }
    double x = 0.0;
#pragma unroll
    for (int kk = SMAX - 1; kk >= 0; --kk) {
        if (kk < s) {
            const double xk = readlane_d(r * myinv, pl[kk]);
            if (mystep < kk) r = fma(-a[kk], xk, r);
            if (lane == kk) x = xk;
        }
    }
    return x;
}

// Lower estimate of ||A^-1||_1 for the factored symmetric A (size s).
// One solve per pass of the loop; `state` follows the steps of the method.
template <int SMAX>
__device__ double inv_norm1_estimate(const double (&a)[SMAX], int mystep, double myinv,
                                     const int *pl, int s, int lane) {
    const bool live = lane < s;
    double x = live ? 1.0 / (double)s : 0.0;
    double est = 0.0, xi = 0.0;
    int state = 1, iter = 0, j = 0;
    for (int pass = 0; pass < 16 && state != 0; ++pass) {
        const double y = lu_solve_lane<SMAX>(x, a, mystep, myinv, pl, s, lane);
        const double sg = (y >= 0.0) ? 1.0 : -1.0;
        if (state == 1) {  // y = A^-1 (1/s): first estimate, then z = A^-T sign(y)
            est = wave_sum(fabs(y));
            xi = live ? sg : 0.0;
            x = xi;
            state = 2;
        } else if (state == 2) {  // y holds z: restart from the unit vector at max |z|
            j = wave_argmax_abs(y, lane, s);
            iter = 2;
            x = (lane == j) ? 1.0 : 0.0;
            state = 3;
        } else if (state == 3) {  // y = A^-1 e_j
            const double old = est;
            est = wave_sum(fabs(y));
            const bool same = __all(!live || sg == xi);
            if (same || est <= old) {
                state = 5;
                x = live ? ((lane & 1) ? -1.0 : 1.0) * (1.0 + (double)lane / (double)(s - 1)) : 0.0;
            } else {
                xi = live ? sg : 0.0;
                x = xi;
                state = 4;
            }
        } else if (state == 4) {  // y holds z = A^-T sign(..)
            const int jlast = j;
            j = wave_argmax_abs(y, lane, s);
            const double zl = readlane_d(fabs(y), jlast), zj = readlane_d(fabs(y), j);
            if (zl != zj && iter < 5) {
                ++iter;
                x = (lane == j) ? 1.0 : 0.0;
                state = 3;
            } else {
                state = 5;
                x = live ? ((lane & 1) ? -1.0 : 1.0) * (1.0 + (double)lane / (double)(s - 1)) : 0.0;
            }
        } else {  // state 5: alternating test vector
            const double t = 2.0 * wave_sum(fabs(y)) / (3.0 * (double)s);
            est = fmax(est, t);
            state = 0;
        }
    }
    return est;
}

// L applied to phi(||x - x_j||) at x_0 = 0, for a stencil node at (x, y).
__device__ __forceinline__ double rhs_phs(double x, double y, int m, int code) {
    const double d2 = x * x + y * y;
    const double r = sqrt(d2);
    if (code == RBF_OP_ID) return ipow(d2, (m - 1) / 2) * r;
    const double rm2 = ipow(d2, (m - 3) / 2) * r;
    if (code == RBF_OP_DX) return (-(double)m * rm2) * x;
    if (code == RBF_OP_DY) return (-(double)m * rm2) * y;
    return (double)(m * m) * rm2;  // Laplacian of r^m in 2-D
}

// L applied to monomial x^a y^b at x_0 = 0.
__device__ __forceinline__ double rhs_poly(int a, int b, int code) {
    if (code == RBF_OP_ID) return (a == 0 && b == 0) ? 1.0 : 0.0;
    if (code == RBF_OP_DX) return (a == 1 && b == 0) ? 1.0 : 0.0;
    if (code == RBF_OP_DY) return (a == 0 && b == 1) ? 1.0 : 0.0;
    return ((a == 2 && b == 0) || (a == 0 && b == 2)) ? 2.0 : 0.0;
}

// Entry (lane, j) of [A P; P^T 0] (0 beyond s) in local coordinates; sx, sy
// hold the scaled stencil offsets of all lanes, (xt, yt) this lane's own,
// (ea, eb) its monomial exponents when n <= lane < s.
__device__ __forceinline__ double system_entry(int lane, int j, int n, int s, int m, double xt,
                                               double yt, int ea, int eb, const double *sx,
                                               const double *sy) {
    if (lane < n) {
        if (j < n) {
            const double ddx = xt - sx[j], ddy = yt - sy[j];
            const double dd = ddx * ddx + ddy * ddy;
            return ipow(dd, (m - 1) / 2) * sqrt(dd);
        }
        if (j < s) {
            int ja, jb;
            mono_exp(j - n, ja, jb);
            return pow_chain(xt, ja) * pow_chain(yt, jb);
        }
        return 0.0;
    }
    if (lane < s && j < n) return pow_chain(sx[j], ea) * pow_chain(sy[j], eb);
    return 0.0;
}

// SMAX bounds the system size; FIXED: the number of operators is exactly
// NOPS (fewer right-hand sides held per lane, no guards on them); COND: the
// condition estimate is computed (a separate instantiation, so that the
// plain solve does not carry its registers).
template <int SMAX, bool FIXED, int NOPS, bool COND>
__global__ void __launch_bounds__(64) k_weights(const double *__restrict__ xq, int64_t nq,
                                                const double *__restrict__ xs, int64_t ns,
                                                const int *__restrict__ idx, int n, int m, int q,
                                                OpSet ops, double *__restrict__ w,
                                                double *__restrict__ cond,
                                                unsigned long long *__restrict__ bad) {
    __shared__ double sx[64], sy[64];
    constexpr int NO = FIXED ? NOPS : kMaxOps;  // right-hand sides held per lane
    __shared__ double sol[NO][SMAX];
    __shared__ int pl[SMAX];

    const int64_t row = blockIdx.x;
    const int lane = threadIdx.x;
    const int kp = (q < 0) ? 0 : (q + 1) * (q + 2) / 2;
    const int s = n + kp;
    const int nops = FIXED ? NOPS : ops.n;

    // 1. Stencil in shifted coordinates; exact power-of-two scaling.
    // A stencil index outside [0, ns) marks the row bad before any load
    // through it (the lane then reads source 0 instead).
    double dx = 0.0, dy = 0.0, d2 = 0.0;
    bool bad_index = false;
    if (lane < n) {
        int j = idx[(int64_t)lane * nq + row];
        if (j < 0 || (int64_t)j >= ns) {
            bad_index = true;
            j = 0;
        }
        dx = xs[j] - xq[row];
        dy = xs[ns + j] - xq[nq + row];
        d2 = dx * dx + dy * dy;
    }
    const double d2max = wave_max(d2);
    int E = 0;
    frexp(d2max, &E);
    const int e = (E >= 0) ? (E + 1) / 2 : -((-E) / 2);
    bool bad_row = !(d2max > 0.0) || !isfinite(d2max) || bad_index;
    const double xt = ldexp(dx, -e), yt = ldexp(dy, -e);
    sx[lane] = xt;
    sy[lane] = yt;
    __syncthreads();

    // 2. This lane's row of [A P; P^T 0] and its right-hand sides.
    int ea = 0, eb = 0;
    if (lane >= n && lane < s) mono_exp(lane - n, ea, eb);
    double a[SMAX], b[NO];
#pragma unroll
    for (int j = 0; j < SMAX; ++j) a[j] = system_entry(lane, j, n, s, m, xt, yt, ea, eb, sx, sy);
    // This lane's right-hand sides (recomputed, not kept, for the
    // refinement's residual).
    auto rhs = [&](int o) {
        if (o >= nops) return 0.0;
        if (lane < n) return rhs_phs(xt, yt, m, ops.code[o]);
        if (lane < s) return rhs_poly(ea, eb, ops.code[o]);
        return 0.0;
    };
#pragma unroll
    for (int o = 0; o < NO; ++o) b[o] = rhs(o);

    // Scale for the singularity test: largest entry of the whole matrix.
    double amax = 0.0;
#pragma unroll
    for (int j = 0; j < SMAX; ++j) amax = fmax(amax, fabs(a[j]));
    amax = wave_max(amax);
    const double tiny = 16.0 * __DBL_EPSILON__ * amax;
    double anorm = 0.0;  // ||A_aug||_1 (largest absolute row sum; A_aug symmetric)
    if constexpr (COND) {
        double rs = 0.0;
#pragma unroll
        for (int j = 0; j < SMAX; ++j) rs += fabs(a[j]);
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) rs = fmax(rs, __shfl_xor(rs, off, 64));
        anorm = readlane_d(rs, 0);
    }

    // 3. LU with partial pivoting across lanes.
    int mystep = (lane < s) ? INT_MAX : -1;  // INT_MAX: row not yet a pivot
    double myinv = 0.0;
#pragma unroll
    for (int kk = 0; kk < SMAX; ++kk) {
        if (kk < s) {
            const int piv = wave_argmax((mystep == INT_MAX) ? fabs(a[kk]) : -1.0, lane);
            const double pv = readlane_d(a[kk], piv);
            if (!(fabs(pv) > tiny) || !isfinite(pv)) bad_row = true;
            const double inv = (pv != 0.0) ? 1.0 / pv : 0.0;
            const bool elim = (mystep == INT_MAX) && lane != piv;
            // Rows that do not eliminate use the multiplier 0: fma(-0, p, a)
            // returns a unchanged for finite p, so no per-entry select.
            const double l = elim ? a[kk] * inv : 0.0;
            if (lane == piv) {
                mystep = kk;
                myinv = inv;
                pl[kk] = lane;
            }
            if (elim) a[kk] = l;  // multiplier, kept for the refinement solve
#pragma unroll
            for (int j = kk + 1; j < SMAX; ++j) a[j] = fma(-l, readlane_d(a[j], piv), a[j]);
#pragma unroll
            for (int o = 0; o < NO; ++o)
                if (o < nops) b[o] = fma(-l, readlane_d(b[o], piv), b[o]);
        }
    }

    // 4. Back substitution: unknown kk lives in the pivot lane of step kk.
#pragma unroll
    for (int kk = SMAX - 1; kk >= 0; --kk) {
        if (kk < s) {
            const int pk = pl[kk];
#pragma unroll
            for (int o = 0; o < NO; ++o) {
                if (o < nops) {
                    const double xk = readlane_d(b[o] * myinv, pk);
                    if (mystep < kk) b[o] = fma(-a[kk], xk, b[o]);
                    if (lane == 0) sol[o][kk] = xk;
                }
            }
        }
    }
    __syncthreads();

    // 5. One refinement step: r = b0 - A0 x in double-FP64, solve with LU.
    // Entries are recomputed (same operations as in step 2) one column at a
    // time; each right-hand side accumulates over j in increasing order.
    double r[NO], hi[NO], lo[NO];
#pragma unroll
    for (int o = 0; o < NO; ++o) {
        hi[o] = rhs(o);
        lo[o] = 0.0;
    }
    if (lane < s) {
#pragma unroll
        for (int j = 0; j < SMAX; ++j) {
            if (j < s) {
                const double aj = system_entry(lane, j, n, s, m, xt, yt, ea, eb, sx, sy);
#pragma unroll
                for (int o = 0; o < NO; ++o) {
                    if (o < nops) {
                        const double xj = sol[o][j];
                        const double p = aj * xj;
                        const double pe = fma(aj, xj, -p);
                        const double t = hi[o] - p;
                        const double bv = t - hi[o];
                        const double err = (hi[o] - (t - bv)) + (-p - bv);
                        hi[o] = t;
                        lo[o] = lo[o] + (err - pe);
                    }
                }
            }
        }
    }
#pragma unroll
    for (int o = 0; o < NO; ++o) r[o] = hi[o] + lo[o];
    // Forward substitution with the stored multipliers (virtual pivoting).
#pragma unroll
    for (int kk = 0; kk < SMAX; ++kk) {
        if (kk < s) {
            const int pk = pl[kk];
#pragma unroll
            for (int o = 0; o < NO; ++o) {
                if (o < nops) {
                    const double yk = readlane_d(r[o], pk);
                    if (mystep > kk && mystep != INT_MAX) r[o] = fma(-a[kk], yk, r[o]);
                }
            }
        }
    }
#pragma unroll
    for (int kk = SMAX - 1; kk >= 0; --kk) {
        if (kk < s) {
            const int pk = pl[kk];
#pragma unroll
            for (int o = 0; o < NO; ++o) {
                if (o < nops) {
                    const double dk = readlane_d(r[o] * myinv, pk);
                    if (mystep < kk) r[o] = fma(-a[kk], dk, r[o]);
                    if (lane == 0) sol[o][kk] += dk;
                }
            }
        }
    }
    __syncthreads();

    // 6. Weights in physical units; NaN for failed rows.
    if (lane < n) {
#pragma unroll
        for (int o = 0; o < NO; ++o) {
            if (o < nops) {
                double v = ldexp(sol[o][lane], -e * ops.order[o]);
                if (!isfinite(v)) bad_row = true;
                w[((int64_t)o * n + lane) * nq + row] = v;
            }
        }
    }
    // A row is bad if any lane saw a problem.
    const bool any_bad = __any(bad_row);
    if constexpr (COND) {
        double c = NAN;
        if (!any_bad) c = anorm * inv_norm1_estimate<SMAX>(a, mystep, myinv, pl, s, lane);
        if (lane == 0) cond[row] = c;
    }
    if (any_bad) {
        if (lane < n) {
            for (int o = 0; o < nops; ++o) w[((int64_t)o * n + lane) * nq + row] = NAN;
        }
        if (lane == 0) atomicMin(bad, (unsigned long long)row);
    }
}

}  // namespace

extern "C" rbf_status rbf_assemble_weights(const double *xq, int64_t nq, const double *xs,
                                           int64_t ns, const int32_t *idx, int32_t k, int32_t m,
                                           int32_t q, uint32_t op_mask, double *w,
                                           double *cond_est, int64_t *bad_row, rbf_stream st_) {
    rbf::clear_error();
    const bool force = (op_mask & RBF_FORCE_SMALL_STENCIL) != 0;
    op_mask &= ~RBF_FORCE_SMALL_STENCIL;
    RBF_ARG(bad_row, "rbf_assemble_weights: bad_row must not be NULL");
    *bad_row = -1;
    RBF_ARG(op_mask != 0 && (op_mask & ~15u) == 0, "rbf_assemble_weights: op_mask must be a non-empty subset of ID|DX|DY|LAP");
    RBF_ARG(q >= -1 && q <= 5, "rbf_assemble_weights: q must be in [-1, 5]");
    RBF_ARG(m >= 1 && m <= 11 && (m % 2) == 1, "rbf_assemble_weights: m must be odd in [1, 11]");
    RBF_ARG((op_mask & ~RBF_OP_ID) == 0 || m >= 3,
            "rbf_assemble_weights: derivative operators need m >= 3 (L phi continuous)");
    const int kp = (q < 0) ? 0 : (q + 1) * (q + 2) / 2;
    RBF_ARG(k >= 1 && k + kp <= 64, "rbf_assemble_weights: need 1 <= k and k + (q+1)(q+2)/2 <= 64");
    RBF_ARG(kp < k, "rbf_assemble_weights: stencil must have more nodes than monomials");
    RBF_ARG(force || q < 0 || k >= (q + 1) * (q + 2),
            "rbf_assemble_weights: k < (q+1)(q+2) violates the stability rule (set RBF_FORCE_SMALL_STENCIL to override)");
    RBF_ARG(ns >= k && nq >= 0 && nq < INT_MAX && ns < INT_MAX, "rbf_assemble_weights: sizes out of range");
    RBF_ARG(xs && (nq == 0 || (xq && idx && w)), "rbf_assemble_weights: NULL pointer");
    if (nq == 0) return RBF_OK;
    OpSet ops{};
    for (int c : {1, 2, 4, 8}) {
        if (op_mask & c) {
            ops.code[ops.n] = c;
            ops.order[ops.n] = (c == 1) ? 0 : (c == 8 ? 2 : 1);
            ++ops.n;
        }
    }
    hipStream_t st = rbf::as_stream(st_);
    unsigned long long *dbad = nullptr;
    RBF_HIP(hipMalloc(&dbad, sizeof(unsigned long long)));
    unsigned long long init = ~0ull;
    rbf_status rc = RBF_OK;
    hipError_t e = hipMemcpyAsync(dbad, &init, sizeof(init), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) {
#define RBF_WLAUNCH(SM, FX, NP)                                                                   \
    do {                                                                                          \
        if (cond_est)                                                                             \
            hipLaunchKernelGGL((k_weights<SM, FX, NP, true>), dim3((uint32_t)nq), dim3(64), 0, st, xq, \
                               nq, xs, ns, idx, k, m, q, ops, w, cond_est, dbad);                 \
        else                                                                                      \
            hipLaunchKernelGGL((k_weights<SM, FX, NP, false>), dim3((uint32_t)nq), dim3(64), 0, st, \
                               xq, nq, xs, ns, idx, k, m, q, ops, w, cond_est, dbad);             \
    } while (0)
        if (k + kp <= 38 && ops.n == 1) RBF_WLAUNCH(38, true, 1);
        else if (k + kp <= 38 && ops.n == 2) RBF_WLAUNCH(38, true, 2);
        else if (k + kp <= 38 && ops.n == 3) RBF_WLAUNCH(38, true, 3);
        else if (k + kp <= 40) RBF_WLAUNCH(40, false, kMaxOps);
        else RBF_WLAUNCH(64, false, kMaxOps);
#undef RBF_WLAUNCH
        e = hipGetLastError();
    }
    unsigned long long hb = ~0ull;
    if (e == hipSuccess) e = hipMemcpyAsync(&hb, dbad, sizeof(hb), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    hipFree(dbad);
    if (e != hipSuccess) {
        rbf::set_error("rbf_assemble_weights: %s", hipGetErrorString(e));
        return RBF_E_DEVICE;
    }
    if (hb != ~0ull) {
        *bad_row = (int64_t)hb;
        rbf::set_error("rbf_assemble_weights: singular or non-finite system, or stencil index outside [0, ns), at row %lld",
                       (long long)hb);
        rc = RBF_E_SINGULAR;
    }
    return rc;
}
