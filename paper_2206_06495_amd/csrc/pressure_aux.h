// Pressure solve on general node sets: flexible GMRES (Saad 1993) right-
// preconditioned by a two-level auxiliary-lattice method.  Included by
// solver.hip inside its anonymous namespace (it uses the solver's Krylov
// helpers, the lattice transforms k_pc_gemm / k_pc_tri and rbf_solver).
//
// System: the row-scaled bordered Poisson operator of eq. (18),
//   A x = S A0 x + u1 c (1^T x),   S the row scale, u1 = S chi, c = vscale,
// A0: D_Lap^PP on interior rows, n . grad on wall rows (see k_build_poisson).
//
// Preconditioner z = B^-1 y (one application; kAuxSweeps smoothing sweeps
// on each side of the lattice correction):
//   x1 = W y, then x1 += W (y - A_s x1)  (kAuxSweeps sweeps from 0)
//                                 W = omega / (l1 norm of A's rows)
//   r1 = y - A_s x1               A_s: the sparse part of A
//   g  = R (S^-1 r1)              R: normalised bilinear restriction of the
//                                 interior-node residuals to the interior
//                                 points of an auxiliary (Ka+1)^2 lattice
//                                 over the nodes' bounding square
//   e  = (L5)^+ (g - lam)         L5: 5-point Laplacian of the lattice with
//                                 one-sided homogeneous Neumann wall rows,
//                                 inverted by the fast transform (DCT-II along
//                                 x, tridiagonal along y); lam = mean of g,
//                                 e of zero mean
//   x2 = x1 + J e + mu            J: bilinear interpolation to the nodes
//                                 (wall lattice values copied inward);
//                                 mu = (lam / c - sum J e) / m carries the
//                                 border's constant (the exact form for the
//                                 bordered operator A0 + chi c 1^T)
//   z  = x2, then z += W (y - A_s z)   (kAuxSweeps post-smoothing sweeps)
// The auxiliary lattice is coarser than the nodes (about two node spacings
// per cell): the smoother removes what the lattice cannot represent, the
// lattice solve removes the smooth error the smoother cannot.  A_s 1 = 0
// (the rows reproduce constants), so mu needs no product.
//
// Precision: T = double (the FP64 solve) or float (mixed precision: each
// restart cycle is one step of iterative refinement whose residual
// b - A x is formed in FP64 from FP64 weights, the cycle itself runs on
// FP32-stored weights, vectors and transforms with FP64 dot products, and
// the correction is added to the FP64 iterate).
//
// FGMRES(mr) with classical Gram-Schmidt (one pass per step, or two when
// the solver enables re-orthogonalisation); the Hessenberg
// column, the Givens rotations and the residual estimate are updated on the
// device by one workgroup per step; the host reads a status block after each
// batch of steps.  All reductions are fixed-order (block partials reduced by
// one workgroup), so a solve is repeatable bit for bit.
#pragma once

constexpr int kFgMax = 30;        // restart length (basis vectors per cycle)
constexpr int kFgChunk = 6;       // dot products accumulated per pass over the rows
// Smoother damping of the l1-Jacobi sweeps: the l1 norms of RBF-FD rows are
// several times their diagonal, so steps up to about 2.4 still damp (FGMRES
// steps per solve at h = 1/100 and 1/200, rtol 1e-12: 111 and 118 at 1.3,
// 86 and 96 at 2.0, 78 and 84 at 2.4, divergent smoothing from 2.8).
constexpr double kAuxOmega = 2.0;
// Border scale of the FGMRES operator relative to the solver's: any scale
// gives the same p~ (the constant is removed afterwards); the solver's own
// scale happens to slow FGMRES (140 against 111 steps at h = 1/100 for 0.1
// or less of it).
constexpr double kAuxBorder = 0.1;
constexpr double kMixedInner = 1e-4;  // mixed: per-cycle residual reduction
// Smoothing sweeps before and after the lattice correction.  Two each cost
// two more products per FGMRES step and cut the steps per solve by about a
// third (h = 1/100, rtol 1e-10: 71 steps with one sweep, 48 with two, 39
// with three).
constexpr int kAuxSweeps = 2;

template <class T>
struct AuxOps {
    const int *idx;
    const T *w;       // [k][m] row-scaled Poisson weights (sparse part of A)
    const T *dinv;    // [m] omega / l1 row norm
    const T *sinv;    // [m] 1 / row scale
    const int *rptr;  // [n*n + 1] restriction rows (interior lattice points)
    const int *rcol;  // node indices
    const T *rval;    // weights, summing to 1 per lattice point
    int64_t m;
    int k;
    // Weight of the second smoothing sweep of each pair relative to the
    // first (chosen at set-up from the spectrum of W A_s, see aux_weight).
    double w2 = 1.0;
};

// FGMRES scalars (device).  Basis vector V_j is stored unnormalised with
// its inverse norm vs[j]; every reader multiplies.
struct FgScal {
    double *vs;      // [mr+1] inverse norms
    double *part;    // [kFgMax + 2][kMaxBlocks] partial sums
    double *h1, *h2; // [mr+1] Gram-Schmidt coefficients of the two passes
    double *hn2;     // [1] ||w||^2 after the last Gram-Schmidt pass
    double *H;       // [(mr+1) * mr] Hessenberg matrix, column-major
    double *cs, *sn; // [mr] Givens rotations
    double *g;       // [mr+1] rotated right-hand side
    double *y;       // [mr] coefficients of the update
    double *resh;    // [mr+1] |g_{j}| per step of the cycle
    double *partZ;   // [kMaxBlocks] sums of J e (interpolated correction)
    double *partO;   // [kMaxBlocks] sums of z (border term of A z)
    double *one;     // [1] = 1.0 (unit scale of an explicit input vector)
    // status, read by the host in one copy: flag, step, then (as doubles)
    // |g_{j+1}| now, 4 steps earlier, the cycle's target, ||b||^2, beta.
    int *flag, *step;
    double *stat;
};

template <class T>
struct FgDev {
    T *V;            // [(mr+1)][m]
    T *Z;            // [mr][m] preconditioned directions
    T *res, *t1;     // [m] preconditioner work
    T *x1, *z1;      // [m] smoothed vectors of the extra sweeps
    T *wd;           // [m] newest basis vector times the smoother diagonal W
    FgScal s;
};

// -------------------------------------------------------------- kernels --
// Row r of A_s applied to the values f(j) at the stencil columns; KT > 0
// fixes the width, its loads issued CH slots at a time (CH divides KT).
// Plain (temporal) loads: the Poisson operator (about 62 MB at h = 1/400)
// and the Krylov vectors of a cycle fit the 256 MB last-level cache
// together and are read several times per FGMRES step (non-temporal loads
// of the operator: 20 us per smoothing product, plain loads: 14.5 us).
template <int KT, int CH, class T, class F>
__device__ __forceinline__ T aux_row(const AuxOps<T> &P, int64_t r, F f) {
    T acc = 0;
    if constexpr (KT > 0) {
        static_assert(KT % CH == 0, "chunk must divide the stencil width");
#pragma unroll
        for (int q0 = 0; q0 < KT; q0 += CH) {
            int jj[CH];
            T ww[CH];
#pragma unroll
            for (int q = 0; q < CH; ++q) jj[q] = *(P.idx + (int64_t)(q0 + q) * P.m + r);
#pragma unroll
            for (int q = 0; q < CH; ++q) ww[q] = *(P.w + (int64_t)(q0 + q) * P.m + r);
#pragma unroll
            for (int q = 0; q < CH; ++q) acc = fma(ww[q], f(jj[q]), acc);
        }
    } else {
        for (int q = 0; q < P.k; ++q)
            acc = fma(P.w[(int64_t)q * P.m + r], f(P.idx[(int64_t)q * P.m + r]), acc);
    }
    return acc;
}

// Two lanes per row for the 28-entry stencils of the smoothing products:
// lanes l and l + 32 of a wave take the two halves of row l's stencil, so a
// launch has twice the waves (and loads in flight) of one lane per row.
constexpr int kRowsPerBlock2 = kThreads / 2;

// This lane's row in the two-lanes-per-row layout (one row pair per thread,
// no grid-stride loop) and the half of the stencil it takes.
__device__ __forceinline__ int64_t row2_of(int &half) {
    const int lane = threadIdx.x & 63;
    half = lane >> 5;
    return (int64_t)rbf::xcd_block(blockIdx.x, gridDim.x) * kRowsPerBlock2 +
           (threadIdx.x >> 6) * 32 + (lane & 31);
}

// Row r of the sparse part applied to f, each lane summing its half of the
// stencil; both lanes of the pair return the row's sum (half 0 + half 1).
template <int KT, class T, class F>
__device__ __forceinline__ T aux_row2(const AuxOps<T> &P, int64_t r, int half, F f) {
    static_assert(KT > 0 && KT % 2 == 0, "two halves of a fixed stencil");
    constexpr int H = KT / 2;
    int jj[H];
    T ww[H];
#pragma unroll
    for (int q = 0; q < H; ++q) jj[q] = P.idx[(int64_t)(half * H + q) * P.m + r];
#pragma unroll
    for (int q = 0; q < H; ++q) ww[q] = P.w[(int64_t)(half * H + q) * P.m + r];
    T acc = 0;
#pragma unroll
    for (int q = 0; q < H; ++q) acc = fma(ww[q], f(jj[q]), acc);
    return acc + __shfl_xor(acc, 32, 64);
}

// Grid of the smoothing products: one row pair per thread for KT > 0, the
// grid-stride row loop otherwise.
template <int KT>
inline dim3 aux_grid(int64_t m, int nb) {
    return (KT > 0) ? dim3(rbf::blocks_for(m, kRowsPerBlock2)) : dim3(nb);
}

// Pre-smoothing sweep from x = W y: x1 = sc (yd + W (y - A_s yd)), y
// scaled by sc = *ys, yd = W y unscaled (one gathered value per neighbour).
template <int KT, class T>
__global__ void __launch_bounds__(kThreads) k_aux_pre(AuxOps<T> P, const T *__restrict__ y,
                                                       const T *__restrict__ yd,
                                                       const double *ys, T *__restrict__ x1,
                                                       const int *flag) {
    if (*flag != 0) return;
    const T sc = (T)*ys;
    if constexpr (KT > 0) {
        int half;
        const int64_t r = row2_of(half);
        const int64_t rr = (r < P.m) ? r : P.m - 1;
        const T ax = aux_row2<KT>(P, rr, half, [&](int j) { return yd[j]; });
        if (half == 0 && r < P.m) x1[r] = sc * (yd[r] + (T)P.w2 * P.dinv[r] * (y[r] - ax));
    } else {
        for (int64_t it = 0;; ++it) {
            const int64_t r = row_of(it);
            if (r - threadIdx.x >= P.m) break;
            if (r < P.m) {
                const T ax = aux_row<KT, 1>(P, r, [&](int j) { return yd[j]; });
                x1[r] = sc * (yd[r] + (T)P.w2 * P.dinv[r] * (y[r] - ax));
            }
        }
    }
}

// Preconditioner stage 1: res = S^-1 (sc y - su A_s u) for the smoothed
// vector su u (u gathered once per neighbour; sc = *ys, su = *us).
template <int KT, class T>
__global__ void __launch_bounds__(kThreads) k_aux_res(AuxOps<T> P, const T *__restrict__ y,
                                                       const double *ys, const T *__restrict__ u,
                                                       const double *us, T *__restrict__ res,
                                                       const int *flag) {
    if (*flag != 0) return;
    const T sc = (T)*ys, su = (T)*us;
    if constexpr (KT > 0) {
        int half;
        const int64_t r = row2_of(half);
        const int64_t rr = (r < P.m) ? r : P.m - 1;
        const T ax = aux_row2<KT>(P, rr, half, [&](int j) { return u[j]; });
        if (half == 0 && r < P.m) res[r] = P.sinv[r] * (sc * y[r] - su * ax);
    } else {
        for (int64_t it = 0;; ++it) {
            const int64_t r = row_of(it);
            if (r - threadIdx.x >= P.m) break;
            if (r < P.m) {
                const T ax = aux_row<KT, 1>(P, r, [&](int j) { return u[j]; });
                res[r] = P.sinv[r] * (sc * y[r] - su * ax);
            }
        }
    }
}

// Power iteration for the largest eigenvalue of W A_s, the smoother's
// operator (set-up only): y = W A_s (s x) and block partial sums of y^2;
// with s = 1 / ||x|| the norm of y estimates the eigenvalue.
template <class T>
__global__ void __launch_bounds__(kThreads) k_aux_power(AuxOps<T> P, const double *__restrict__ x,
                                                         double s, double *__restrict__ y,
                                                         double *part) {
    double acc[1] = {0.0};
    for (int64_t it = 0;; ++it) {
        const int64_t r = row_of(it);
        if (r - threadIdx.x >= P.m) break;
        if (r < P.m) {
            const double ax = (double)aux_row<0, 1>(P, r, [&](int j) { return (T)x[j]; });
            const double v = s * (double)P.dinv[r] * ax;
            y[r] = v;
            acc[0] += v * v;
        }
    }
    store_partials<1>(acc, part, gridDim.x);
}

// Start vector of the power iteration: a fixed hash pattern in [-1, 1).
__global__ void k_aux_power_start(int64_t m, double *__restrict__ x) {
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= m) return;
    const uint32_t hsh = (uint32_t)r * 2654435761u;
    x[r] = (double)(hsh >> 8) * (1.0 / 8388608.0) - 1.0;
}

// yd = W y for an explicit input vector.
template <class T>
__global__ void k_aux_scale(AuxOps<T> P, const T *__restrict__ y, T *__restrict__ yd) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < P.m;
         r += (int64_t)gridDim.x * blockDim.x)
        yd[r] = y[r] * P.dinv[r];
}

// Stage 2: restriction to the interior lattice points, X(q) = sum rval res
// (about 18 entries per point with two node spacings per cell): 4 lanes per
// point take every 4th entry, then combine in a fixed order.
template <class T>
__global__ void __launch_bounds__(256) k_aux_restrict(AuxOps<T> P, Lat L,
                                                       const T *__restrict__ res, int nq) {
    if (*L.flag != 0) return;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int q = t >> 2, sub = t & 3;
    double g = 0.0;
    if (q < nq) {
        const int e1 = P.rptr[q + 1];
        for (int e = P.rptr[q] + sub; e < e1; e += 4)
            g += (double)P.rval[e] * (double)res[P.rcol[e]];
    }
    g += __shfl_xor(g, 1, 64);
    g += __shfl_xor(g, 2, 64);
    if (q < nq && sub == 0) lat_store(L, L.X, q, g);
}

// Lattice value of the transform solve (Z, column-major in X) at lattice
// node (i, j); wall nodes take their inward neighbour's value (homogeneous
// one-sided Neumann rows).
__device__ __forceinline__ double aux_lattice(const Lat &L, int i, int j) {
    const int ci = min(max(i, 1), L.K - 1), cj = min(max(j, 1), L.K - 1);
    return lat_load(L, L.X, (int64_t)(ci - 1) + (int64_t)(cj - 1) * L.n);
}

// Stage 3: t1 = W y + J e (W y from yd), and block sums of J e.
template <class T>
__global__ void __launch_bounds__(kThreads) k_aux_interp(AuxOps<T> P, Lat L,
                                                          const T *__restrict__ u,
                                                          const double *us, T *__restrict__ t1,
                                                          double *partZ) {
    if (*L.flag != 0) return;
    const T su = (T)*us;
    const int K1 = L.K + 1;
    double acc[1] = {0.0};
    for (int64_t it = 0;; ++it) {
        const int64_t r = row_of(it);
        if (r - threadIdx.x >= P.m) break;
        if (r < P.m) {
            const int c = L.cell[r];
            const int i0 = c % K1, j0 = c / K1;
            const double fx = L.fx[r], fy = L.fy[r];
            const double z = (1.0 - fy) * ((1.0 - fx) * aux_lattice(L, i0, j0) +
                                           fx * aux_lattice(L, i0 + 1, j0)) +
                             fy * ((1.0 - fx) * aux_lattice(L, i0, j0 + 1) +
                                   fx * aux_lattice(L, i0 + 1, j0 + 1));
            t1[r] = su * u[r] + (T)z;
            acc[0] += z;
        }
    }
    store_partials<1>(acc, partZ, gridDim.x);
}

// Stage 4: z = t1 + mu + W (y - A_s t1) (MU: the border's constant mu is
// added; later sweeps add none); block sums of z (border term of the
// product that follows).  A_s mu = 0: the rows reproduce constants.
template <int KT, class T, bool MU>
__global__ void __launch_bounds__(kThreads) k_aux_post(AuxOps<T> P, Lat L,
                                                        const T *__restrict__ y, const double *ys,
                                                        const T *__restrict__ t1,
                                                        const double *partZ,
                                                        T *__restrict__ z, double *partO) {
    if (*L.flag != 0) return;
    double mu = 0.0;
    if constexpr (MU) {
        double sz[1];
        load_partials<1>(partZ, gridDim.x, sz);
        mu = (*L.mean / L.c - sz[0]) / (double)P.m;
    }
    const T sc = (T)*ys;
    double acc[1] = {0.0};
    for (int64_t it = 0;; ++it) {
        const int64_t r = row_of(it);
        if (r - threadIdx.x >= P.m) break;
        if (r < P.m) {
            const T at = aux_row<KT, (KT > 0 ? KT : 1)>(P, r, [&](int j) { return t1[j]; });
            const T zr = t1[r] + (T)mu + (MU ? (T)1 : (T)P.w2) * P.dinv[r] * (sc * y[r] - at);
            z[r] = zr;
            acc[0] += (double)zr;
        }
    }
    store_partials<1>(acc, partO, gridDim.x);
}

// The same sweep for 28-entry stencils with two lanes per row: blocks of
// 2 kThreads threads on the same grid and rows per block as k_aux_post, so
// the block sums of z keep their count.
template <class T, bool MU>
__global__ void __launch_bounds__(2 * kThreads) __attribute__((amdgpu_waves_per_eu(4)))
k_aux_post2(AuxOps<T> P, Lat L,
                                                           const T *__restrict__ y,
                                                           const double *ys,
                                                           const T *__restrict__ t1,
                                                           const double *partZ,
                                                           T *__restrict__ z, double *partO) {
    if (*L.flag != 0) return;
    __shared__ double lds[2 * kThreads / 64];
    const int lane = threadIdx.x & 63, half = lane >> 5, wv = threadIdx.x >> 6;
    const int nb = gridDim.x;  // <= kMaxBlocks = 2 blockDim.x: two partials per thread
    // The partials of mu and the first row iteration's product (every block
    // has one) are loaded before mu is reduced, so that the reduction
    // overlaps the gathers.
    const double pz0 = (MU && (int)threadIdx.x < nb) ? partZ[threadIdx.x] : 0.0;
    const double pz1 =
        (MU && (int)threadIdx.x + 2 * kThreads < nb) ? partZ[threadIdx.x + 2 * kThreads] : 0.0;
    const int64_t bx = rbf::xcd_block(blockIdx.x, nb);
    int64_t r = bx * kThreads + wv * 32 + (lane & 31);
    int64_t rr = (r < P.m) ? r : P.m - 1;
    T at = aux_row2<28>(P, rr, half, [&](int j) { return t1[j]; });
    double mu = 0.0;
    if constexpr (MU) {
        double sz[1] = {pz0 + pz1};
        rbf::block_sum<1>(sz, lds);
        mu = (*L.mean / L.c - sz[0]) / (double)P.m;
    }
    const T sc = (T)*ys;
    double acc[1] = {0.0};
#pragma unroll 1
    for (int64_t it = 0;; ++it) {
        if ((bx + it * nb) * kThreads >= P.m) break;
        if (it > 0) {
            r = (bx + it * nb) * kThreads + wv * 32 + (lane & 31);
            rr = (r < P.m) ? r : P.m - 1;
            at = aux_row2<28>(P, rr, half, [&](int j) { return t1[j]; });
        }
        if (half == 0 && r < P.m) {
            const T zr = t1[r] + (T)mu + (MU ? (T)1 : (T)P.w2) * P.dinv[r] * (sc * y[r] - at);
            z[r] = zr;
            acc[0] += (double)zr;
        }
    }
    rbf::block_sum<1>(acc, lds);
    if (threadIdx.x == 0) partO[blockIdx.x] = acc[0];
}

// Cycle start: r = b - A x in FP64 (FP64 weights and border), V_0 = r and
// W V_0; block sums of ||r||^2 and ||b||^2 (rows 0 and 1 of part).
template <int KT, class T>
__global__ void __launch_bounds__(kThreads) k_fg_init(EllM A, const double *__restrict__ b,
                                                       const double *__restrict__ x,
                                                       const double *partX, T *__restrict__ V0,
                                                       const T *__restrict__ dinv,
                                                       T *__restrict__ wd, double *part) {
    const int nb = gridDim.x;
    double sx[1] = {0.0};
    if (A.u1) load_partials<1>(partX, nb, sx);
    double acc[2] = {0.0, 0.0};
    for (int64_t it = 0;; ++it) {
        const int64_t r = row_of(it);
        if (r - threadIdx.x >= A.n) break;
        if (r < A.n) {
            double ax[1][1] = {};
            const double *ws[1] = {A.w};
            rbf::ell_row<KT, 1>(A.idx, ws, A.n, r, A.k, GatherN<1>{x, A.n}, ax);
            const double u1 = A.u1 ? A.u1[r] * A.vscale : 0.0;
            const double rr = b[r] - (ax[0][0] + u1 * sx[0]);
            V0[r] = (T)rr;
            wd[r] = (T)rr * dinv[r];
            acc[0] += rr * rr;
            acc[1] += b[r] * b[r];
        }
    }
    double v0[1] = {acc[0]}, v1[1] = {acc[1]};
    store_partials<1>(v0, part, nb);
    store_partials<1>(v1, part + kMaxBlocks, nb);
}

// Reduce nq rows of nb block partials (row q at q * kMaxBlocks) into
// out[q]: one workgroup per row, a fixed order.  GATE: exit when the flag
// is set (inside an Arnoldi step).
template <bool GATE>
__global__ void __launch_bounds__(256) k_fg_reduce(const double *part, int nb, int nq,
                                                   double *out, const int *flag) {
    if (GATE && *flag != 0) return;
    const int q = blockIdx.x;
    double v[1] = {0.0};
    for (int b = threadIdx.x; b < nb; b += 256) v[0] += part[(int64_t)q * kMaxBlocks + b];
    __shared__ double lds[4];
    rbf::block_sum<1>(v, lds);
    if (threadIdx.x == 0) out[q] = v[0];
}

// Cycle start, one thread: beta = ||r||, the cycle's target (FP64:
// tol ||b||; mixed: also kMixedInner beta), convergence of the true
// residual (flag 1), g = beta e_1.  red: {||r||^2, ||b||^2}; ||b|| is
// taken from the first cycle.
__global__ void k_fg_start(FgScal F, const double *red, double tol, int mixed, int first) {
    const double rr = red[0], bbv = first ? red[1] : F.stat[3];
    const double beta = sqrt(rr);
    const double goal = tol * sqrt(fmax(bbv, 1e-300));
    F.step[0] = 0;
    F.stat[0] = beta;
    F.stat[1] = beta;
    F.stat[3] = bbv;
    F.stat[4] = beta;
    F.resh[0] = beta;
    if (!isfinite(beta)) {
        F.flag[0] = -1;
        return;
    }
    if (beta <= goal || beta == 0.0) {
        F.flag[0] = 1;
        return;
    }
    F.stat[2] = mixed ? fmax(goal, kMixedInner * beta) : goal;
    F.vs[0] = 1.0 / beta;
    F.g[0] = beta;
    F.flag[0] = 0;
}

// Block partial dots (V_i vs_i, w) for i <= j, kFgChunk at a time; w is
// this thread's rows of the new vector (re-read per chunk).
template <class T>
__device__ __forceinline__ void fg_dots(const T *V, const double *vs, const T *w, int64_t m, int j,
                                        double *part) {
#pragma unroll 1
    for (int i0 = 0; i0 <= j; i0 += kFgChunk) {
        double acc[kFgChunk];
#pragma unroll
        for (int c = 0; c < kFgChunk; ++c) acc[c] = 0.0;
#pragma unroll 1
        for (int64_t it = 0;; ++it) {
            const int64_t r = row_of(it);
            if (r - threadIdx.x >= m) break;
            if (r < m) {
                const double wr = (double)w[r];
#pragma unroll
                for (int c = 0; c < kFgChunk; ++c)
                    if (i0 + c <= j) acc[c] += (double)V[(int64_t)(i0 + c) * m + r] * wr;
            }
        }
#pragma unroll
        for (int c = 0; c < kFgChunk; ++c) acc[c] *= (i0 + c <= j) ? vs[i0 + c] : 0.0;
        __shared__ double lds[kFgChunk * (kThreads / 64)];
        rbf::block_sum<kFgChunk>(acc, lds);
        if (threadIdx.x == 0)
            for (int c = 0; c < kFgChunk && i0 + c <= j; ++c)
                part[(int64_t)(i0 + c) * kMaxBlocks + blockIdx.x] = acc[c];
    }
}

// Arnoldi step j, product: w = A z_j (sparse part in T plus the border with
// sum z_j from partO; u1 must not be null), stored in V[j+1]; block partial
// dots (V_i vs_i, w).
template <int KT, class T>
__global__ void __launch_bounds__(kThreads) k_fg_av(AuxOps<T> P, const double *__restrict__ u1,
                                                     double vscale, FgDev<T> F, int j) {
    if (*F.s.flag != 0) return;
    double sz[1];
    load_partials<1>(F.s.partO, gridDim.x, sz);
    const double bterm = vscale * sz[0];  // border: u1 c (1^T z)
    const T *z = F.Z + (int64_t)j * P.m;
    T *w = F.V + (int64_t)(j + 1) * P.m;
#pragma unroll 1
    for (int64_t it = 0;; ++it) {
        const int64_t r = row_of(it);
        if (r - threadIdx.x >= P.m) break;
        if (r < P.m) {
            const T az = aux_row<KT, (KT > 0 ? KT : 1)>(P, r, [&](int c) { return z[c]; });
            w[r] = (T)((double)az + u1[r] * bterm);
        }
    }
    fg_dots(F.V, F.s.vs, w, P.m, j, F.s.part);
}

// The same step for 28-entry stencils with two lanes per row: blocks of
// 2 kThreads threads on the same grid (and the same kThreads rows per block
// and grid-stride iteration), so the partial sums keep their count; lanes l
// and l + 32 of a wave take the two halves of row l's stencil.  The dots are
// taken in the same pass over the rows: lane l + 32 h multiplies w by the
// basis vectors i = 2c + h (slot c), so that each vector is read once, and
// the slots are summed per half-wave by DPP, then over the waves in a fixed
// order.
constexpr int kAvThreads = 2 * kThreads;
constexpr int kFgSlots = (kFgMax + 1) / 2;  // basis vectors per half-wave

// Slot sums in LDS: column wv of lds (2 kFgSlots rows of NW) holds wave
// wv's running sums of the basis vectors i = 2c (half 0) and 2c + 1
// (half 1), owned by the wave's lane 0.  fg_slot_add adds one pass's
// products (half-wave sums by DPP; every lane must be active);
// fg_slot_partials sums the waves in a fixed order and writes the block
// partials of rows i <= j of part, scaled by vs_i.
template <int NW>
__device__ __forceinline__ void fg_slot_zero(int ns, double *lds) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0)
        for (int i = 0; i < 2 * ns; ++i) lds[i * NW + wv] = 0.0;
}

template <int NW>
__device__ __forceinline__ void fg_slot_add(const double (&prod)[kFgSlots], int ns, double *lds) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < kFgSlots; ++c) {
        if (c < ns) {
            double se, so;
            rbf::half_wave_sums(prod[c], se, so);
            if (lane == 0) {
                lds[(2 * c) * NW + wv] += se;
                lds[(2 * c + 1) * NW + wv] += so;
            }
        }
    }
}

template <int NW>
__device__ __forceinline__ void fg_slot_partials(int j, const double *vs, double *part,
                                                 const double *lds) {
    __syncthreads();
    if ((int)threadIdx.x <= j) {
        const int q = threadIdx.x;
        double t = 0.0;
#pragma unroll
        for (int v = 0; v < NW; ++v) t += lds[q * NW + v];
        part[(int64_t)q * kMaxBlocks + blockIdx.x] = t * vs[q];
    }
}

template <class T>
__global__ void __launch_bounds__(kAvThreads) __attribute__((amdgpu_waves_per_eu(4))) k_fg_av2(AuxOps<T> P, const double *__restrict__ u1,
                                                       double vscale, FgDev<T> F, int j) {
    if (*F.s.flag != 0) return;
    constexpr int NW = kAvThreads / 64;
    __shared__ double lds[2 * kFgSlots * NW];
    const int lane = threadIdx.x & 63, half = lane >> 5, wv = threadIdx.x >> 6;
    const int nb = gridDim.x;  // <= kMaxBlocks = 2 blockDim.x: two partials per thread
    const T *z = F.Z + (int64_t)j * P.m;
    T *w = F.V + (int64_t)(j + 1) * P.m;
    // The partials of 1^T z and the first row iteration's product (every
    // block has one) are loaded before the border sum is reduced, so that
    // the reduction overlaps the gathers.
    const double po0 = ((int)threadIdx.x < nb) ? F.s.partO[threadIdx.x] : 0.0;
    const double po1 =
        ((int)threadIdx.x + kAvThreads < nb) ? F.s.partO[threadIdx.x + kAvThreads] : 0.0;
    const int64_t bx = rbf::xcd_block(blockIdx.x, nb);
    int64_t r = bx * kThreads + wv * 32 + (lane & 31);
    int64_t rr = (r < P.m) ? r : P.m - 1;
    T az = aux_row2<28>(P, rr, half, [&](int c) { return z[c]; });
    double sz[1] = {po0 + po1};
    rbf::block_sum<1>(sz, lds);
    const double bterm = vscale * sz[0];  // border: u1 c (1^T z)
    const int ns = (j + 2) >> 1;
    fg_slot_zero<NW>(ns, lds);
#pragma unroll 1
    for (int64_t it = 0;; ++it) {
        if ((bx + it * nb) * kThreads >= P.m) break;
        if (it > 0) {
            r = (bx + it * nb) * kThreads + wv * 32 + (lane & 31);
            rr = (r < P.m) ? r : P.m - 1;
            az = aux_row2<28>(P, rr, half, [&](int c) { return z[c]; });
        }
        const T wt = (T)((double)az + u1[rr] * bterm);
        // The basis is read after the product, so that the two sets of
        // loads in flight do not share the registers.  Slot c of half 1
        // reads V[j+1] (this row of w, not yet stored) when 2c + 1 > j; that
        // value is not used.
        __builtin_amdgcn_sched_barrier(0);
        const T *Vh = F.V + (int64_t)half * P.m + rr;
        const double wr = (r < P.m) ? (double)wt : 0.0;
        double prod[kFgSlots];
#pragma unroll
        for (int c = 0; c < kFgSlots; ++c) {
            prod[c] = 0.0;
            if (c < ns) {
                const double v = (double)Vh[(int64_t)(2 * c) * P.m];
                if (2 * c + half <= j) prod[c] = v * wr;
            }
        }
        if (half == 0 && r < P.m) w[r] = wt;
        fg_slot_add<NW>(prod, ns, lds);
    }
    fg_slot_partials<NW>(j, F.s.vs, F.s.part, lds);
}

// Gram-Schmidt update w -= sum_i h_i vs_i V_i (i <= j).  PASS 1 (the first
// of two passes): then block partial dots (V_i vs_i, w) for the second;
// PASS 2 (the last pass, the only one by default): then block partial
// ||w||^2, and W w for the next preconditioner application.
// Blocks of 2 kThreads threads on the kThreads-rows grid: lanes l and l + 32
// of a wave share row l, each reading the basis vectors of one parity
// (slot c: i = 2c + h), which serve both the update and, in PASS 1, the
// dots with the updated w.
template <class T, int PASS>
__global__ void __launch_bounds__(2 * kThreads) __attribute__((amdgpu_waves_per_eu(4))) k_fg_gs(FgDev<T> F, const double *h,
                                                         const T *__restrict__ dinv, int64_t m,
                                                         int j) {
    if (*F.s.flag != 0) return;
    constexpr int NW = 2 * kThreads / 64;
    __shared__ double c[kFgMax + 1];
    __shared__ double lds[2 * kFgSlots * NW];
    for (int i = threadIdx.x; i <= j; i += blockDim.x) c[i] = h[i] * F.s.vs[i];
    __syncthreads();
    const int lane = threadIdx.x & 63, half = lane >> 5, wv = threadIdx.x >> 6;
    const int nb = gridDim.x;
    const int ns = (j + 2) >> 1;
    const int64_t bx = rbf::xcd_block(blockIdx.x, nb);
    T *w = F.V + (int64_t)(j + 1) * m;
    double nrm[1] = {0.0};
    if constexpr (PASS == 1) fg_slot_zero<NW>(ns, lds);
#pragma unroll 1
    for (int64_t it = 0;; ++it) {
        if ((bx + it * nb) * kThreads >= m) break;
        const int64_t r = (bx + it * nb) * kThreads + wv * 32 + (lane & 31);
        const int64_t rr = (r < m) ? r : m - 1;
        // Slot q of half 1 reads V[j+1] = w when 2q + 1 > j (not used).
        const T *Vh = F.V + (int64_t)half * m + rr;
        double vv[kFgSlots];
#pragma unroll
        for (int q = 0; q < kFgSlots; ++q) vv[q] = (q < ns) ? (double)Vh[(int64_t)(2 * q) * m] : 0.0;
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < kFgSlots; ++q)
            if (q < ns && 2 * q + half <= j) s += c[2 * q + half] * vv[q];
        s += __shfl_xor(s, 32, 64);
        const T wt = (T)((double)w[rr] - s);
        if (half == 0 && r < m) {
            w[r] = wt;
            if constexpr (PASS == 2) F.wd[r] = wt * dinv[r];
            nrm[0] += (double)wt * (double)wt;
        }
        if constexpr (PASS == 1) {
            const double wr = (r < m) ? (double)wt : 0.0;
            double prod[kFgSlots];
#pragma unroll
            for (int q = 0; q < kFgSlots; ++q)
                prod[q] = (q < ns && 2 * q + half <= j) ? vv[q] * wr : 0.0;
            fg_slot_add<NW>(prod, ns, lds);
        }
    }
    if constexpr (PASS == 1) {
        fg_slot_partials<NW>(j, F.s.vs, F.s.part, lds);
    } else {
        rbf::block_sum<1>(nrm, lds);
        if (threadIdx.x == 0) F.s.part[blockIdx.x] = nrm[0];
    }
}

// Arnoldi step j, one workgroup: Hessenberg column j = h1 + h2 with
// H(j+1, j) = ||w||, previous rotations applied, a new rotation, the
// residual estimate |g_{j+1}| and the status (4: the cycle's target met or
// an exact breakdown; 3: the cycle is full; -1: non-finite).
// ||w||^2 is reduced here from the block partials of k_fg_gs<2> (row 0 of
// part, nb blocks), in the order k_fg_reduce uses.
__global__ void __launch_bounds__(256) k_fg_tail(FgScal F, int j, int mr, int nb) {
    if (*F.flag != 0) return;
    __shared__ double col[kFgMax + 1], cs[kFgMax], sn[kFgMax];
    const int lane = threadIdx.x;
    double v[1] = {0.0};
    for (int b = lane; b < nb; b += 256) v[0] += F.part[b];
    __shared__ double lds[4];
    rbf::block_sum<1>(v, lds);
    for (int i = lane; i <= j; i += 256) {
        col[i] = F.h1[i] + F.h2[i];
        if (i < j) {
            cs[i] = F.cs[i];
            sn[i] = F.sn[i];
        }
    }
    __syncthreads();
    if (lane != 0) return;
    double *Hc = F.H + (int64_t)j * (mr + 1);
    F.hn2[0] = v[0];
    const double hn = sqrt(v[0]);
    col[j + 1] = hn;
    for (int i = 0; i < j; ++i) {
        const double a = col[i], b = col[i + 1];
        col[i] = cs[i] * a + sn[i] * b;
        col[i + 1] = -sn[i] * a + cs[i] * b;
    }
    const double a = col[j], b = col[j + 1];
    const double den = hypot(a, b);
    const double c = (den > 0.0) ? a / den : 1.0, s = (den > 0.0) ? b / den : 0.0;
    F.cs[j] = c;
    F.sn[j] = s;
    col[j] = den;
    for (int i = 0; i <= j; ++i) Hc[i] = col[i];
    Hc[j + 1] = 0.0;
    const double gj = F.g[j];
    F.g[j] = c * gj;
    F.g[j + 1] = -s * gj;
    const double res = fabs(s * gj);
    F.vs[j + 1] = (hn > 0.0) ? 1.0 / hn : 0.0;
    F.resh[j + 1] = res;
    F.step[0] = j + 1;
    F.stat[0] = res;
    F.stat[1] = F.resh[max(0, j + 1 - 4)];
    if (!isfinite(res) || !isfinite(den)) F.flag[0] = -1;
    else if (res <= F.stat[2] || hn == 0.0 || den == 0.0) F.flag[0] = 4;
    else if (j + 1 >= mr) F.flag[0] = 3;
}

// End of a cycle of nstep steps, one thread: back substitution H y = g.
__global__ void __launch_bounds__(256) k_fg_solve(FgScal F, int nstep, int mr) {
    __shared__ double Hs[kFgMax * kFgMax], gs[kFgMax], ys[kFgMax];
    for (int e = threadIdx.x; e < nstep * nstep; e += blockDim.x) {
        const int l = e / nstep, i = e % nstep;  // column l, row i
        Hs[l * kFgMax + i] = F.H[(int64_t)l * (mr + 1) + i];
    }
    for (int i = threadIdx.x; i < nstep; i += blockDim.x) gs[i] = F.g[i];
    __syncthreads();
    if (threadIdx.x != 0) return;
    for (int i = nstep - 1; i >= 0; --i) {
        double s = gs[i];
        for (int l = i + 1; l < nstep; ++l) s -= Hs[l * kFgMax + i] * ys[l];
        const double d = Hs[i * kFgMax + i];
        ys[i] = (d != 0.0) ? s / d : 0.0;
    }
    for (int i = 0; i < nstep; ++i) F.y[i] = ys[i];
}

// x += sum_i y_i Z_i (FP64 iterate).
template <class T>
__global__ void __launch_bounds__(kThreads) k_fg_x(const T *__restrict__ Z, const double *ycoef,
                                                    int nstep, int64_t m, double *__restrict__ x) {
    for (int64_t r = blockIdx.x * (int64_t)kThreads + threadIdx.x; r < m;
         r += (int64_t)gridDim.x * kThreads) {
        double s = x[r];
        for (int i = 0; i < nstep; ++i) s += ycoef[i] * (double)Z[(int64_t)i * m + r];
        x[r] = s;
    }
}

// l1 row norms of the stored Poisson rows: dinv = omega / sum |w|, and
// 1 / row scale.
__global__ void k_aux_rows(int64_t m, int k, const double *__restrict__ w,
                           const double *__restrict__ rs, double *dinv, double *sinv) {
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= m) return;
    double s = 0.0;
    for (int q = 0; q < k; ++q) s += fabs(w[(int64_t)q * m + r]);
    dinv[r] = (s > 0.0) ? kAuxOmega / s : 0.0;
    sinv[r] = 1.0 / rs[r];
}

// FP32 copies for the mixed-precision cycles.
__global__ void k_aux_to_f32(int64_t n, const double *__restrict__ a, float *__restrict__ b) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        b[i] = (float)a[i];
}
