// rbf_assemble_weights: batched local PHS+poly RBF-FD weight solves.
//
// Sec. 2.1 (eqs. (3)-(9)): for evaluation node x_0 with stencil x_1..x_n,
//   [A P; P^T 0] [w; c] = [L phi; L P],  A_ij = ||x_i - x_j||^m,
// P_jt = the monomials of degree <= q at x_j, right-hand sides L applied to
// phi(||x - x_j||) and to the monomials at x = x_0; w is kept.
//
// The paper's stencil (n = 28, cubic polynomials) without the condition
// estimate goes to k_weights_pair (two systems per wavefront, further
// below); every other form to k_weights:
// one wavefront (64 lanes) solves one system.  Lane i owns row i of the
// augmented matrix (s = n + K_p <= 64 rows) in registers; the monomials of
// the P block are computed once per stencil node and shared through LDS.
// LU with partial pivoting runs across lanes: the pivot is found by one
// unsigned maximum reduction over the wave (the lane number packed into the
// low bits of a key made of the value's high word), the pivot lane writes
// the rest of its row to LDS, every lane reads it as broadcasts and every
// other unfinished row eliminates with it (row swaps are virtual: each lane
// remembers the step at which its row became pivot).  The residual of the
// refinement step recomputes the lane's row of the original matrix (a copy
// in LDS would cost more in occupancy than the recomputation).  All
// right-hand sides (one per operator) are eliminated together.  One step of
// iterative refinement with a residual accumulated in double-FP64
// arithmetic (exact products via fma) brings the solution to within a few
// ulps of the exact solution of the FP64 system.
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

// Cross-lane maximum without LDS traffic: DPP moves inside each 16-lane
// row (rotations by 8 and 4, then quad swaps of 2 and 1 leave every lane of
// a row with the row's result), then the four rows' results read by
// v_readlane and combined uniformly.  Exact maxima, so the reduction order
// does not matter.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

constexpr int kDppRor8 = 0x128, kDppRor4 = 0x124, kDppSwap2 = 0x4E, kDppSwap1 = 0xB1;

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

// Lane whose row was chosen as pivot at elimination step kk (wave-uniform):
// exactly one lane holds mystep == kk once the factorisation is done.
__device__ __forceinline__ int step_lane(int mystep, int kk) {
    const unsigned long long m = __ballot(mystep == kk);
    return m ? __builtin_ctzll(m) : 0;
}

// Solve A x = r with the factors of k_weights' LU: lane i holds r_i and
// receives x_i (0 beyond s).  a holds the multipliers of the steps that
// eliminated this lane's row (steps before mystep) and its row of U (steps
// after it); the masks turn the entries of the other factor into zero
// multipliers instead of selecting results.
template <int SMAX>
__device__ __forceinline__ double lu_solve_lane(double r, const double (&a)[SMAX], int mystep,
                                                double myinv, int s, int lane) {
#pragma unroll
    for (int kk = 0; kk < SMAX; ++kk) {
        if (kk < s) {
            const double lk = (mystep > kk && mystep != INT_MAX) ? a[kk] : 0.0;
            r = fma(-lk, readlane_d(r, step_lane(mystep, kk)), r);
        }
    }
    double x = 0.0;
#pragma unroll
    for (int kk = SMAX - 1; kk >= 0; --kk) {
        if (kk < s) {
            const double uk = (mystep < kk) ? a[kk] : 0.0;
            const double xk = readlane_d(r * myinv, step_lane(mystep, kk));
            r = fma(-uk, xk, r);
            if (lane == kk) x = xk;
        }
    }
    return x;
}

// Lower estimate of ||A^-1||_1 for the factored symmetric A (size s).
// One solve per pass of the loop; `state` follows the steps of the method.
template <int SMAX>
__device__ double inv_norm1_estimate(const double (&a)[SMAX], int mystep, double myinv, int s,
                                     int lane) {
    const bool live = lane < s;
    double x = live ? 1.0 / (double)s : 0.0;
    double est = 0.0, xi = 0.0;
    int state = 1, iter = 0, j = 0;
    for (int pass = 0; pass < 16 && state != 0; ++pass) {
        const double y = lu_solve_lane<SMAX>(x, a, mystep, myinv, s, lane);
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

// Lane of the largest c >= 0 over the wave (lanes with c < 0 or NaN are not
// candidates), up to a relative 2^-14: the key is the high word of c (sign,
// exponent, 20 mantissa bits) with its low six bits replaced by 63 - lane,
// so one unsigned maximum reduction yields a lane whose value is within
// 2^-14 of the largest (ties in the key go to the lowest lane).  Partial
// pivoting needs no more: the multipliers stay below 1 + 2^-14.
__device__ __forceinline__ int wave_argmax_packed(double c, int lane) {
    const unsigned hi = (unsigned)((unsigned long long)__double_as_longlong(c) >> 32);
    unsigned key = (c >= 0.0) ? ((hi & ~63u) | (unsigned)(63 - lane)) : 0u;
    key = max(key, (unsigned)__builtin_amdgcn_update_dpp(0, (int)key, kDppRor8, 0xF, 0xF, false));
    key = max(key, (unsigned)__builtin_amdgcn_update_dpp(0, (int)key, kDppRor4, 0xF, 0xF, false));
    key = max(key, (unsigned)__builtin_amdgcn_update_dpp(0, (int)key, kDppSwap2, 0xF, 0xF, false));
    key = max(key, (unsigned)__builtin_amdgcn_update_dpp(0, (int)key, kDppSwap1, 0xF, 0xF, false));
    const unsigned k0 = (unsigned)__builtin_amdgcn_readlane((int)key, 0);
    const unsigned k1 = (unsigned)__builtin_amdgcn_readlane((int)key, 16);
    const unsigned k2 = (unsigned)__builtin_amdgcn_readlane((int)key, 32);
    const unsigned k3 = (unsigned)__builtin_amdgcn_readlane((int)key, 48);
    return 63 - (int)(max(max(k0, k1), max(k2, k3)) & 63u);
}

// SMAX bounds the system size; FIXED: the number of operators is exactly
// NOPS (fewer right-hand sides held per lane, no guards on them); COND: the
// condition estimate is computed (a separate instantiation, so that the
// plain solve does not carry its registers).
template <int SMAX, bool FIXED, int NOPS, bool COND>
__device__ __forceinline__ void weights_system(const double *__restrict__ xq, int64_t nq,
                                                const double *__restrict__ xs, int64_t ns,
                                                const int *__restrict__ idx, int n, int m, int q,
                                                OpSet ops, double *__restrict__ w,
                                                double *__restrict__ cond,
                                                unsigned long long *__restrict__ bad) {
    // Right-hand sides held per lane; those beyond the operator count are
    // zero and stay zero, so the loops run over all NO without guards.
    constexpr int NO = FIXED ? NOPS : kMaxOps;
    // k_p < n and n + k_p <= SMAX bound the monomial count by SMAX / 2.
    constexpr int KPS = (SMAX / 2 < 21) ? SMAX / 2 : 21;
    static_assert(SMAX <= 64, "one row per lane");
    __shared__ double sx[64], sy[64];
    __shared__ double smono[KPS][SMAX];     // monomial t at stencil node i < n
    __shared__ double prow[2][SMAX + NO];   // pivot row of a step (alternate buffers)
    __shared__ double sol[NO][SMAX];
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
    // The monomials of this lane's node: slot t has fixed exponents, so the
    // products fold to straight-line code; the P block reads them back.
    if (lane < n) {
#pragma unroll
        for (int t = 0; t < KPS; ++t) {
            if (t < kp) {
                int ta, tb;
                mono_exp(t, ta, tb);
                smono[t][lane] = pow_chain(xt, ta) * pow_chain(yt, tb);
            }
        }
    }
    __syncthreads();

    // 2. This lane's row of [A P; P^T 0] and its right-hand sides.  Entry
    // (lane, j) for j < s (0 for lanes >= s); the branches on j are uniform.
    const int tl = (lane >= n && lane < s) ? lane - n : 0;  // P^T row: monomial slot
    const int nl = (lane < n) ? lane : 0;
    auto entry = [&](int j) -> double {
        if (j < n) {
            const double ddx = xt - sx[j], ddy = yt - sy[j];
            const double dd = ddx * ddx + ddy * ddy;
            const double phi = ipow(dd, (m - 1) / 2) * sqrt(dd);
            const double pt = smono[tl][j];
            return (lane < n) ? phi : ((lane < s) ? pt : 0.0);
        }
        const double pj = smono[j - n][nl];
        return (lane < n) ? pj : 0.0;
    };
    int ea = 0, eb = 0;
    if (lane >= n && lane < s) mono_exp(lane - n, ea, eb);
    double a[SMAX], b[NO];
#pragma unroll
    for (int j = 0; j < SMAX; ++j) a[j] = (j < s) ? entry(j) : 0.0;
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

    // 3. LU with partial pivoting across lanes.  The pivot lane writes the
    // rest of its row and its right-hand sides to LDS; every lane reads them
    // as broadcasts (two buffers, so one barrier per step orders the reads of
    // a step before the writes two steps later).
    int mystep = (lane < s) ? INT_MAX : -1;  // INT_MAX: row not yet a pivot
    double myinv = 0.0;
#pragma unroll
    for (int kk = 0; kk < SMAX; ++kk) {
        if (kk < s) {
            double *pr = prow[kk & 1];
            const int piv = wave_argmax_packed((mystep == INT_MAX) ? fabs(a[kk]) : -1.0, lane);
            if (lane == piv) {
                if (mystep != INT_MAX) bad_row = true;  // no candidate left (non-finite column)
                mystep = kk;
#pragma unroll
                for (int j = kk; j < SMAX; ++j) pr[j] = a[j];
#pragma unroll
                for (int o = 0; o < NO; ++o) pr[SMAX + o] = b[o];
            }
            __syncthreads();
            const double pv = pr[kk];
            if (!(fabs(pv) > tiny) || !isfinite(pv)) bad_row = true;
            // 1 / pv: hardware reciprocal and two Newton steps (a last-bit
            // error here is removed by the refinement step).
            double inv = 0.0;
            if (pv != 0.0) {
                double x = __builtin_amdgcn_rcp(pv);
                x = fma(x, fma(-pv, x, 1.0), x);
                inv = fma(x, fma(-pv, x, 1.0), x);
            }
            if (lane == piv) myinv = inv;
            const bool elim = (mystep == INT_MAX);
            // Rows that do not eliminate use the multiplier 0: fma(-0, p, a)
            // returns a unchanged for finite p, so no per-entry select.
            const double l = elim ? a[kk] * inv : 0.0;
            if (elim) a[kk] = l;  // multiplier, kept for the refinement solve
#pragma unroll
            for (int j = kk + 1; j < SMAX; ++j) a[j] = fma(-l, pr[j], a[j]);
#pragma unroll
            for (int o = 0; o < NO; ++o) b[o] = fma(-l, pr[SMAX + o], b[o]);
        }
    }

    // 4. Back substitution: unknown kk lives in the pivot lane of step kk.
#pragma unroll
    for (int kk = SMAX - 1; kk >= 0; --kk) {
        if (kk < s) {
            const int pk = step_lane(mystep, kk);
            const double uk = (mystep < kk) ? a[kk] : 0.0;
#pragma unroll
            for (int o = 0; o < NO; ++o) {
                const double xk = readlane_d(b[o] * myinv, pk);
                b[o] = fma(-uk, xk, b[o]);
                if (lane == 0) sol[o][kk] = xk;
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
#pragma unroll
    for (int j = 0; j < SMAX; ++j) {
        if (j < s) {
            const double aj = entry(j);
#pragma unroll
            for (int o = 0; o < NO; ++o) {
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
#pragma unroll
    for (int o = 0; o < NO; ++o) r[o] = hi[o] + lo[o];
    // Forward substitution with the stored multipliers (virtual pivoting).
#pragma unroll
    for (int kk = 0; kk < SMAX; ++kk) {
        if (kk < s) {
            const int pk = step_lane(mystep, kk);
            const double lk = (mystep > kk && mystep != INT_MAX) ? a[kk] : 0.0;
#pragma unroll
            for (int o = 0; o < NO; ++o) r[o] = fma(-lk, readlane_d(r[o], pk), r[o]);
        }
    }
#pragma unroll
    for (int kk = SMAX - 1; kk >= 0; --kk) {
        if (kk < s) {
            const int pk = step_lane(mystep, kk);
            const double uk = (mystep < kk) ? a[kk] : 0.0;
#pragma unroll
            for (int o = 0; o < NO; ++o) {
                const double dk = readlane_d(r[o] * myinv, pk);
                r[o] = fma(-uk, dk, r[o]);
                if (lane == 0) sol[o][kk] += dk;
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
        if (!any_bad) c = anorm * inv_norm1_estimate<SMAX>(a, mystep, myinv, s, lane);
        if (lane == 0) cond[row] = c;
    }
    if (any_bad) {
        if (lane < n) {
            for (int o = 0; o < nops; ++o) w[((int64_t)o * n + lane) * nq + row] = NAN;
        }
        if (lane == 0) atomicMin(bad, (unsigned long long)row);
    }
}

// The plain solve for systems of at most 40 rows is compiled for four waves
// per SIMD (at most 128 VGPRs, a few of them spilled to scratch): the extra
// wave hides more of the latency of the elimination steps than three waves
// without spills.  The other forms keep the compiler's own register budget.
template <int SMAX, bool FIXED, int NOPS>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4)))
k_weights(const double *__restrict__ xq, int64_t nq, const double *__restrict__ xs, int64_t ns,
          const int *__restrict__ idx, int n, int m, int q, OpSet ops, double *__restrict__ w,
          double *__restrict__ cond, unsigned long long *__restrict__ bad) {
    weights_system<SMAX, FIXED, NOPS, false>(xq, nq, xs, ns, idx, n, m, q, ops, w, cond, bad);
}

template <int SMAX, bool FIXED, int NOPS, bool COND>
__global__ void __launch_bounds__(64)
k_weights_any(const double *__restrict__ xq, int64_t nq, const double *__restrict__ xs, int64_t ns,
              const int *__restrict__ idx, int n, int m, int q, OpSet ops, double *__restrict__ w,
              double *__restrict__ cond, unsigned long long *__restrict__ bad) {
    weights_system<SMAX, FIXED, NOPS, COND>(xq, nq, xs, ns, idx, n, m, q, ops, w, cond, bad);
}

// ---------------------------------------------------------------------------
// Two systems per wavefront for the paper's stencil (n = 28 nodes, cubic
// polynomials, K_p = 10): lanes 0-31 solve system 2b, lanes 32-63 system
// 2b + 1, lane l of a half owning row l of the RBF block A.  Block
// elimination of [A P; P^T 0] [w; c] = [f; g]:
//   LU of A with partial pivoting (rows of the half) carried through the
//   columns [P | f], back substitution gives X = A^-1 P and y = A^-1 f;
//   the Schur system S c = P^T y - g with S = P^T X (10 x 10) is formed by
//   dot products over LDS and solved with partial pivoting; w = y - X c.
// One refinement step as in the one-system kernel: the residual of the
// whole saddle-point system in double-FP64 (entries recomputed), then the
// same block solve for the correction.  A and the augmented matrix have
// comparable condition numbers on these stencils and S is far better
// conditioned, so the block order loses nothing the refinement does not
// recover.
constexpr int kPairN = 28, kPairKP = 10;

// Largest v within each 32-lane half (every lane gets its half's value).
__device__ __forceinline__ double half_max(double v, int lane) {
    v = fmax(v, dpp_d<kDppRor8>(v));
    v = fmax(v, dpp_d<kDppRor4>(v));
    v = fmax(v, dpp_d<kDppSwap2>(v));
    v = fmax(v, dpp_d<kDppSwap1>(v));
    const double h0 = fmax(readlane_d(v, 0), readlane_d(v, 16));
    const double h1 = fmax(readlane_d(v, 32), readlane_d(v, 48));
    return (lane < 32) ? h0 : h1;
}

// Pivot key of a candidate c >= 0 (0: no candidate): the high word of c
// with its low six bits replaced by 63 - lane, as in wave_argmax_packed.
__device__ __forceinline__ unsigned pivot_key(double c, bool cand, int lane) {
    const unsigned hi = (unsigned)((unsigned long long)__double_as_longlong(c) >> 32);
    return (cand && c >= 0.0) ? ((hi & ~63u) | (unsigned)(63 - lane)) : 0u;
}

// Lane of the largest key within each half; the half's idle lane 31 when
// no lane of the half is a candidate.
__device__ __forceinline__ int half_argmax_key(unsigned key, int lane) {
    key = max(key, (unsigned)__builtin_amdgcn_update_dpp(0, (int)key, kDppRor8, 0xF, 0xF, false));
    key = max(key, (unsigned)__builtin_amdgcn_update_dpp(0, (int)key, kDppRor4, 0xF, 0xF, false));
    key = max(key, (unsigned)__builtin_amdgcn_update_dpp(0, (int)key, kDppSwap2, 0xF, 0xF, false));
    key = max(key, (unsigned)__builtin_amdgcn_update_dpp(0, (int)key, kDppSwap1, 0xF, 0xF, false));
    const unsigned h0 = max((unsigned)__builtin_amdgcn_readlane((int)key, 0),
                            (unsigned)__builtin_amdgcn_readlane((int)key, 16));
    const unsigned h1 = max((unsigned)__builtin_amdgcn_readlane((int)key, 32),
                            (unsigned)__builtin_amdgcn_readlane((int)key, 48));
    const unsigned km = (lane < 32) ? h0 : h1;
    return km ? 63 - (int)(km & 63u) : (lane & 32) + 31;
}

// 1 / p: hardware reciprocal and two Newton steps (0 for p = 0).
__device__ __forceinline__ double recip_nr(double p) {
    if (p == 0.0) return 0.0;
    double x = __builtin_amdgcn_rcp(p);
    x = fma(x, fma(-p, x, 1.0), x);
    return fma(x, fma(-p, x, 1.0), x);
}

// hi + lo -= a * x, exactly rounded product and compensated sum (the
// refinement residual's double-FP64 accumulation).
__device__ __forceinline__ void dd_sub_prod(double &hi, double &lo, double a, double x) {
    const double p = a * x;
    const double pe = fma(a, x, -p);
    const double t = hi - p;
    const double bv = t - hi;
    const double err = (hi - (t - bv)) + (-p - bv);
    hi = t;
    lo = lo + (err - pe);
}

template <int NO>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2)))
k_weights_pair(const double *__restrict__ xq, int64_t nq, const double *__restrict__ xs,
               int64_t ns, const int *__restrict__ idx, int m, OpSet ops,
               double *__restrict__ w, unsigned long long *__restrict__ bad) {
    constexpr int N = kPairN, KP = kPairKP, R = KP + NO;
    __shared__ double sx[2][32], sy[2][32];
    __shared__ double prow[2][2][N + R];  // [buffer][half] pivot row of a step
    __shared__ double sz[2][N][R];        // [half][unknown] X = A^-1 P | y = A^-1 f
    __shared__ double sp[2][N][KP];       // [half][node] monomials
    __shared__ double ss[2][KP][R];       // [half] rows of [S | P^T y - g]
    __shared__ double sc[2][KP][NO];      // [half] c (then its correction)
    __shared__ double sw[2][N][NO];       // [half] w
    __shared__ double sr[2][KP][NO];      // [half] constraint residuals, then S right-hand sides
    const int lane = threadIdx.x, h = lane >> 5, l = lane & 31;
    const int64_t row = (int64_t)blockIdx.x * 2 + h;
    const bool valid = row < nq;
    const bool live = valid && l < N;
    const int ln = (l < N) ? l : N - 1;   // stand-in row index for idle lanes
    const int lk = (l < KP) ? l : KP - 1;

    // 1. Stencil offsets, exact power-of-two scaling per system.
    double dx = 0.0, dy = 0.0, d2 = 0.0;
    bool bad_row = false;
    if (live) {
        int j = idx[(int64_t)l * nq + row];
        if (j < 0 || (int64_t)j >= ns) {
            bad_row = true;
            j = 0;
        }
        dx = xs[j] - xq[row];
        dy = xs[ns + j] - xq[nq + row];
        d2 = dx * dx + dy * dy;
    }
    const double d2max = half_max(d2, lane);
    int E = 0;
    frexp(d2max, &E);
    const int e = (E >= 0) ? (E + 1) / 2 : -((-E) / 2);
    if (valid && (!(d2max > 0.0) || !isfinite(d2max))) bad_row = true;
    const double xt = ldexp(dx, -e), yt = ldexp(dy, -e);
    sx[h][l] = xt;
    sy[h][l] = yt;
    // This node's monomials (fixed exponents per slot), kept in LDS.
#pragma unroll
    for (int t = 0; t < KP; ++t) {
        int ta, tb;
        mono_exp(t, ta, tb);
        if (l < N) sp[h][l][t] = pow_chain(xt, ta) * pow_chain(yt, tb);
    }
    __syncthreads();

    // 2. Row l of A (recomputed the same way for the residual), of P, and of f.
    auto phi = [&](int j) {
        const double ddx = xt - sx[h][j], ddy = yt - sy[h][j];
        const double dd = ddx * ddx + ddy * ddy;
        return ipow(dd, (m - 1) / 2) * sqrt(dd);
    };
    auto rhsf = [&](int o) { return live ? rhs_phs(xt, yt, m, ops.code[o]) : 0.0; };
    auto rhsg = [&](int t, int o) {
        int ta, tb;
        mono_exp(t, ta, tb);
        return rhs_poly(ta, tb, ops.code[o]);
    };
    double a[N], pc[KP], b[NO];
    double amax = 0.0;
#pragma unroll
    for (int j = 0; j < N; ++j) {
        a[j] = live ? phi(j) : 0.0;
        amax = fmax(amax, fabs(a[j]));
    }
#pragma unroll
    for (int t = 0; t < KP; ++t) {
        pc[t] = live ? sp[h][ln][t] : 0.0;
        amax = fmax(amax, fabs(pc[t]));
    }
#pragma unroll
    for (int o = 0; o < NO; ++o) b[o] = rhsf(o);
    const double tiny = 16.0 * __DBL_EPSILON__ * half_max(amax, lane);

    // 3. LU of A with partial pivoting over the half's rows, carried through
    // [P | f]; the pivot row goes through LDS (two buffers, one barrier per
    // step).
    int mystep = live ? INT_MAX : -1;
    double myinv = 0.0;
#pragma unroll
    for (int kk = 0; kk < N; ++kk) {
        double *pr = prow[kk & 1][h];
        const int piv = half_argmax_key(pivot_key(fabs(a[kk]), mystep == INT_MAX, lane), lane);
        if (lane == piv) {
            if (mystep != INT_MAX) bad_row = true;  // no candidate left in this column
            mystep = kk;
#pragma unroll
            for (int j = kk; j < N; ++j) pr[j] = a[j];
#pragma unroll
            for (int t = 0; t < KP; ++t) pr[N + t] = pc[t];
#pragma unroll
            for (int o = 0; o < NO; ++o) pr[N + KP + o] = b[o];
        }
        __syncthreads();
        const double pv = pr[kk];
        if (!(fabs(pv) > tiny) || !isfinite(pv)) bad_row = true;
        const double inv = recip_nr(pv);
        if (lane == piv) myinv = inv;
        const bool elim = (mystep == INT_MAX);
        const double lm = elim ? a[kk] * inv : 0.0;
        if (elim) a[kk] = lm;
#pragma unroll
        for (int j = kk + 1; j < N; ++j) a[j] = fma(-lm, pr[j], a[j]);
#pragma unroll
        for (int t = 0; t < KP; ++t) pc[t] = fma(-lm, pr[N + t], pc[t]);
#pragma unroll
        for (int o = 0; o < NO; ++o) b[o] = fma(-lm, pr[N + KP + o], b[o]);
    }

    // 4. Back substitution: unknown kk is solved in the pivot lane of step
    // kk, which stores row kk of [X | y] in LDS for the other lanes.
#pragma unroll
    for (int kk = N - 1; kk >= 0; --kk) {
        if (mystep == kk) {
#pragma unroll
            for (int t = 0; t < KP; ++t) sz[h][kk][t] = pc[t] * myinv;
#pragma unroll
            for (int o = 0; o < NO; ++o) sz[h][kk][KP + o] = b[o] * myinv;
        }
        __syncthreads();
        const double uk = (mystep < kk) ? a[kk] : 0.0;
#pragma unroll
        for (int t = 0; t < KP; ++t) pc[t] = fma(-uk, sz[h][kk][t], pc[t]);
#pragma unroll
        for (int o = 0; o < NO; ++o) b[o] = fma(-uk, sz[h][kk][KP + o], b[o]);
    }

    // 5. [S | P^T y - g] by dot products over the nodes, 32 entries a round.
#pragma unroll 1
    for (int e0 = 0; e0 < KP * R; e0 += 32) {
        const int en = e0 + l;
        const int ec = (en < KP * R) ? en : 0;
        const int t = ec / R, c = ec - t * R;
        double acc = 0.0;
#pragma unroll 4
        for (int j = 0; j < N; ++j) acc = fma(sp[h][j][t], sz[h][j][c], acc);
        if (c >= KP) acc -= rhsg(t, c - KP);
        if (en < KP * R) ss[h][t][c] = acc;
    }
    __syncthreads();

    // 6. S c = P^T y - g: lanes 0..KP-1 of each half own the rows.
    double srow[R];
#pragma unroll
    for (int c = 0; c < R; ++c) srow[c] = (l < KP) ? ss[h][lk][c] : 0.0;
    int mys = (valid && l < KP) ? INT_MAX : -1;
    double sinv = 0.0;
    auto s_factor = [&]() {
#pragma unroll
        for (int kk = 0; kk < KP; ++kk) {
            double *pr = prow[kk & 1][h];
            const int piv = half_argmax_key(pivot_key(fabs(srow[kk]), mys == INT_MAX, lane), lane);
            if (lane == piv) {
                if (mys != INT_MAX) bad_row = true;
                mys = kk;
#pragma unroll
                for (int c = kk; c < R; ++c) pr[c] = srow[c];
            }
            __syncthreads();
            const double pv = pr[kk];
            if (!(pv != 0.0) || !isfinite(pv)) bad_row = true;
            const double inv = recip_nr(pv);
            if (lane == piv) sinv = inv;
            const bool elim = (mys == INT_MAX);
            const double lm = elim ? srow[kk] * inv : 0.0;
            if (elim) srow[kk] = lm;
#pragma unroll
            for (int c = kk + 1; c < R; ++c) srow[c] = fma(-lm, pr[c], srow[c]);
        }
    };
    s_factor();
    // Back substitution of the S system into sc (right-hand sides in
    // srow[KP..]); S's factors stay in srow[0..KP-1] for the correction.
    auto s_back = [&](double (&rs)[NO]) {
#pragma unroll
        for (int kk = KP - 1; kk >= 0; --kk) {
            if (mys == kk) {
#pragma unroll
                for (int o = 0; o < NO; ++o) sc[h][kk][o] = rs[o] * sinv;
            }
            __syncthreads();
            const double uk = (mys < kk) ? srow[kk] : 0.0;
#pragma unroll
            for (int o = 0; o < NO; ++o) rs[o] = fma(-uk, sc[h][kk][o], rs[o]);
        }
    };
    double rs[NO];
#pragma unroll
    for (int o = 0; o < NO; ++o) rs[o] = srow[KP + o];
    s_back(rs);
    __syncthreads();

    // 7. w = y - X c for node l.
    double wv[NO];
#pragma unroll
    for (int o = 0; o < NO; ++o) {
        double s = sz[h][ln][KP + o];
#pragma unroll
        for (int t = 0; t < KP; ++t) s = fma(-sz[h][ln][t], sc[h][t][o], s);
        wv[o] = s;
        if (l < N) sw[h][l][o] = s;
    }
    __syncthreads();

    // 8. Residual of the saddle-point system in double-FP64: RBF rows in
    // lanes 0..N-1, constraint rows (t, o) in lanes t * NO + o.
    double r[NO];
    {
        double hi[NO], lo[NO];
#pragma unroll
        for (int o = 0; o < NO; ++o) {
            hi[o] = rhsf(o);
            lo[o] = 0.0;
        }
#pragma unroll 2
        for (int j = 0; j < N; ++j) {
            const double aj = live ? phi(j) : 0.0;
#pragma unroll
            for (int o = 0; o < NO; ++o) dd_sub_prod(hi[o], lo[o], aj, sw[h][j][o]);
        }
#pragma unroll
        for (int t = 0; t < KP; ++t) {
            const double pt = live ? sp[h][ln][t] : 0.0;
#pragma unroll
            for (int o = 0; o < NO; ++o) dd_sub_prod(hi[o], lo[o], pt, sc[h][t][o]);
        }
#pragma unroll
        for (int o = 0; o < NO; ++o) r[o] = hi[o] + lo[o];
    }
    {
        const int en = (l < KP * NO) ? l : 0;
        const int t = en / NO, o = en - t * NO;
        double hi = rhsg(t, o), lo = 0.0;
#pragma unroll 4
        for (int j = 0; j < N; ++j) dd_sub_prod(hi, lo, sp[h][j][t], sw[h][j][o]);
        __syncthreads();  // every lane has read sc and sw
        if (l < KP * NO) sr[h][t][o] = hi + lo;
    }

    // 9. Correction: y' = A^-1 r (stored factors), S c' = P^T y' - r_c,
    // w' = y' - X c'.
#pragma unroll
    for (int kk = 0; kk < N; ++kk) {
        double *pr = prow[kk & 1][h];
        if (mystep == kk) {
#pragma unroll
            for (int o = 0; o < NO; ++o) pr[o] = r[o];
        }
        __syncthreads();
        const double lkk = (mystep > kk && mystep != INT_MAX) ? a[kk] : 0.0;
#pragma unroll
        for (int o = 0; o < NO; ++o) r[o] = fma(-lkk, pr[o], r[o]);
    }
#pragma unroll
    for (int kk = N - 1; kk >= 0; --kk) {
        if (mystep == kk) {
#pragma unroll
            for (int o = 0; o < NO; ++o) sz[h][kk][KP + o] = r[o] * myinv;
        }
        __syncthreads();
        const double uk = (mystep < kk) ? a[kk] : 0.0;
#pragma unroll
        for (int o = 0; o < NO; ++o) r[o] = fma(-uk, sz[h][kk][KP + o], r[o]);
    }
    {
        const int en = (l < KP * NO) ? l : 0;
        const int t = en / NO, o = en - t * NO;
        double acc = -sr[h][t][o];
#pragma unroll 4
        for (int j = 0; j < N; ++j) acc = fma(sp[h][j][t], sz[h][j][KP + o], acc);
        __syncthreads();  // every lane has read sr
        if (l < KP * NO) sr[h][t][o] = acc;
    }
    __syncthreads();
    // Forward substitution with S's multipliers, then back substitution.
#pragma unroll
    for (int o = 0; o < NO; ++o) rs[o] = (l < KP) ? sr[h][lk][o] : 0.0;
#pragma unroll
    for (int kk = 0; kk < KP; ++kk) {
        double *pr = prow[kk & 1][h];
        if (mys == kk) {
#pragma unroll
            for (int o = 0; o < NO; ++o) pr[o] = rs[o];
        }
        __syncthreads();
        const double lkk = (mys > kk && mys != INT_MAX) ? srow[kk] : 0.0;
#pragma unroll
        for (int o = 0; o < NO; ++o) rs[o] = fma(-lkk, pr[o], rs[o]);
    }
    s_back(rs);
    __syncthreads();

    // 10. Weights in physical units; NaN for failed systems.
    const unsigned long long bm = __ballot(bad_row);
    const bool any_bad = valid && ((h ? (bm >> 32) : (bm & 0xffffffffull)) != 0);
    bool nonfinite = false;
#pragma unroll
    for (int o = 0; o < NO; ++o) {
        double s = sz[h][ln][KP + o];
#pragma unroll
        for (int t = 0; t < KP; ++t) s = fma(-sz[h][ln][t], sc[h][t][o], s);
        const double v = ldexp(wv[o] + s, -e * ops.order[o]);
        if (!isfinite(v)) nonfinite = true;
        if (live) w[((int64_t)o * N + l) * nq + row] = any_bad ? NAN : v;
    }
    const unsigned long long nm = __ballot(live && nonfinite);
    const bool half_nonfinite = (h ? (nm >> 32) : (nm & 0xffffffffull)) != 0;
    if (valid && half_nonfinite && !any_bad && live) {
#pragma unroll
        for (int o = 0; o < NO; ++o) w[((int64_t)o * N + l) * nq + row] = NAN;
    }
    if (valid && (any_bad || half_nonfinite) && l == 0) atomicMin(bad, (unsigned long long)row);
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
            hipLaunchKernelGGL((k_weights_any<SM, FX, NP, true>), dim3((uint32_t)nq), dim3(64), 0, \
                               st, xq, nq, xs, ns, idx, k, m, q, ops, w, cond_est, dbad);         \
        else if constexpr (SM <= 40)                                                              \
            hipLaunchKernelGGL((k_weights<SM, FX, NP>), dim3((uint32_t)nq), dim3(64), 0, st, xq,   \
                               nq, xs, ns, idx, k, m, q, ops, w, cond_est, dbad);                 \
        else                                                                                      \
            hipLaunchKernelGGL((k_weights_any<SM, FX, NP, false>), dim3((uint32_t)nq), dim3(64), 0, \
                               st, xq, nq, xs, ns, idx, k, m, q, ops, w, cond_est, dbad);         \
    } while (0)
        // The paper's stencil without the condition estimate: two systems
        // per wavefront.
        const bool pair = !cond_est && k == kPairN && q == 3 && ops.n >= 1 && ops.n <= 3;
        const dim3 pgrid((uint32_t)((nq + 1) / 2)), pblock(64);
        if (pair && ops.n == 1)
            hipLaunchKernelGGL(k_weights_pair<1>, pgrid, pblock, 0, st, xq, nq, xs, ns, idx, m, ops, w, dbad);
        else if (pair && ops.n == 2)
            hipLaunchKernelGGL(k_weights_pair<2>, pgrid, pblock, 0, st, xq, nq, xs, ns, idx, m, ops, w, dbad);
        else if (pair)
            hipLaunchKernelGGL(k_weights_pair<3>, pgrid, pblock, 0, st, xq, nq, xs, ns, idx, m, ops, w, dbad);
        else if (k + kp <= 38 && ops.n == 1) RBF_WLAUNCH(38, true, 1);
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
