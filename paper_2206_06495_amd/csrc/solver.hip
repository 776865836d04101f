// Fractional-step Navier-Stokes solver on staggered nodes (Sec. 3):
//   stage 1  AB2 advection (eqs. (14)-(15))            k_advect
//   stage 2  Crank-Nicolson viscous step (eq. (16))    k_helm_rhs, k_wall_rhs,
//            with Kim-Moin wall values (eq. (21))      Jacobi sweeps or BiCGSTAB
//                                                      on H (2 RHS)
//   stage 3  divergence (eq. (17)), pressure Poisson   k_divergence,
//            (eq. (18)), pressure (eq. (19)) and       BiCGSTAB on the Poisson
//            velocity correction (eq. (20))            matrix, k_pressure, k_correct
//
// The paper factors its implicit matrices once by LU.  Here the systems are
// solved iteratively on the ELL operators: the pressure by BiCGSTAB (van der
// Vorst 1992) right-preconditioned by a lattice fast-Poisson solve when the
// P-nodes form a jittered lattice, the viscous system by Jacobi sweeps when
// H is strongly diagonally dominant, else by Jacobi-preconditioned BiCGSTAB.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <string>
#include <system_error>
#include <thread>
#include <type_traits>
#include <utility>
#include <vector>

#include <hip/hip_ext.h>

#include "common.h"
#include "dgemm_mfma.h"
#include "ell.h"

namespace {

constexpr int kThreads = 256;
constexpr int kMaxBlocks = 1024;
constexpr int kMaxNR = 2;

// ------------------------------------------------------------ gathers --
template <int NR>
struct GatherN {
    static constexpr int NV = NR;
    const double *x;
    int64_t stride;
    __device__ __forceinline__ void operator()(int j, double (&v)[NR]) const {
#pragma unroll
        for (int c = 0; c < NR; ++c) v[c] = x[c * stride + j];
    }
};

struct Gather2 {
    static constexpr int NV = 2;
    const double *a, *b;
    __device__ __forceinline__ void operator()(int j, double (&v)[2]) const {
        v[0] = a[j];
        v[1] = b[j];
    }
};

// -------------------------------------------------------- reductions --
// Block-partial sums: part[(q * NR + c) * nb + block] for NQ quantities.
template <int NQ>
__device__ __forceinline__ void store_partials(double (&v)[NQ], double *part, int nb) {
    __shared__ double lds[NQ * (kThreads / 64)];
    rbf::block_sum<NQ>(v, lds);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) part[(int64_t)q * nb + blockIdx.x] = v[q];
    }
}

// Each block re-reduces NQ rows of nb partials in a fixed order.
template <int NQ>
__device__ __forceinline__ void load_partials(const double *part, int nb, double (&out)[NQ]) {
    __shared__ double lds[NQ * (kThreads / 64)];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        double s = 0.0;
        for (int b = threadIdx.x; b < nb; b += blockDim.x) s += part[(int64_t)q * nb + b];
        out[q] = s;
    }
    rbf::block_sum<NQ>(out, lds);
}

// ------------------------------------------------------ Krylov state --
// BiCGSTAB (van der Vorst 1992), right-preconditioned with D^-1 (Jacobi when
// JAC, else the identity), for NR right-hand sides sharing every matrix read,
// restructured into two SpMV kernels per iteration.  Used for the pressure
// solve without the lattice preconditioner (NR = 1, identity on the
// row-scaled Poisson matrix); the viscous solve has its own kernels
// (k_h_*, below).
//   k_kry_a(i): at every row, finish the update of iteration i-1
//                 s = r - alpha v,  r' = s - omega t,  x += alpha D^-1 p + omega D^-1 s,
//               start iteration i
//                 p' = r' + beta (p - omega v),  v' = A D^-1 p'
//               where the gathered D^-1 p'_j of the SpMV is recomputed at each
//               neighbour from r, v, t, p (no separate vector pass).
//   k_kry_b(i): alpha = rho / (rh, v'),  t = A D^-1 (r' - alpha v').
// The scalars use (rh, s) = 0, so rho_{i+1} = (rh, r') = -omega (rh, t).
// r, p, v are double-buffered (the kernel that rewrites them also gathers
// the old values at neighbouring rows).  Every scalar is reduced on the
// device from block partial sums written by the producer and re-reduced, in
// a fixed order, by each block of the consumer: deterministic, no host
// round trip.  Convergence (||r'|| <= tol ||b||, tested in k_kry_b) and
// breakdown are device flags that the host reads every few iterations;
// kernels launched after they are set exit at once.
//
// rec[(i * NR + c) * 4 + {0,1,2,3}] = rho_i, alpha_i, omega_i, ||r_i||^2.
// flag[c]: 0 running, 1 converged, -1 non-finite, 2 breakdown (the host
// restarts from the current iterate with rh = r).
// The iteration vectors are interleaved per node, q[j] = {r_0..r_{NR-1},
// v_0.., t_0.., p_0..} (4 NR doubles), so the on-the-fly gathers of the two
// SpMV kernels read one contiguous 16-byte-aligned record per neighbour.
struct KDev {
    double *q[2];                // [n][4 NR], ping-pong by iteration parity
    double *rh;                  // [NR][n]
    double *partA[2];            // 5 quantities x NR x blocks (k_kry_a / init)
    double *partB;               // 4 quantities x NR x blocks (k_kry_b)
    double *partX;               // NR x blocks (sum of x for the rank-one term)
    double *rec, *bb, *rhrh;     // per-iteration scalars, ||b||^2, ||rh||^2
    int *flag, *iters;
};

// Breakdown threshold for |rho| = |(rh, r)| relative to ||rh|| ||r||.
constexpr double kBreakdown = 1e-13;

// A = ELL(idx, w) + u1 (vscale 1^T): the optional rank-one term carries the
// zero-mean border of the pressure-Poisson system (u1 == nullptr: none).
struct EllM {
    const int *idx;
    const double *w;
    const double *dinv;  // nullptr: no preconditioner
    int64_t n;
    int k;
    const double *u1;
    double vscale;
};

// Block sums of NR stacked vectors (for the rank-one term).
template <int NR>
__global__ void __launch_bounds__(kThreads) k_sum(int64_t n, const double *__restrict__ x,
                                                   double *part) {
    double acc[NR] = {};
    for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kThreads) {
#pragma unroll
        for (int c = 0; c < NR; ++c) acc[c] += x[c * n + i];
    }
    store_partials<NR>(acc, part, gridDim.x);
}

// y = x - mean(x) (one right-hand side), the mean from k_sum partials.
__global__ void __launch_bounds__(kThreads) k_sub_mean(int64_t n, const double *part, int nbprev,
                                                        const double *x, double *y) {
    double sm[1];
    load_partials<1>(part, nbprev, sm);
    const double mean = sm[0] / (double)n;
    for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kThreads)
        y[i] = x[i] - mean;
}

__device__ __forceinline__ int64_t row_of(int64_t it) {
    return ((int64_t)rbf::xcd_block(blockIdx.x, gridDim.x) + it * gridDim.x) * kThreads +
           threadIdx.x;
}

__device__ __forceinline__ bool all_done(const int *flag, int nr) {
    for (int c = 0; c < nr; ++c)
        if (flag[c] == 0) return false;
    return true;
}

// partA layout: quantity q in {0: (rh,v'), 1: ||r'||^2, 2: sum r', 3: sum p', 4: sum v'}
// (init: 0: ||r0||^2 (= rho_0), 1: ||r0||^2, 2: sum r0, 3: ||b||^2, 4: 0).
// partB layout: {0: (t,s), 1: (t,t), 2: (rh,t), 3: sum t}.

// r0 = b - A x (x from the caller), rh = r0, p = v = t = 0.
template <int NR, int KT>
__global__ void __launch_bounds__(kThreads) k_kry_init(EllM A, const double *__restrict__ b,
                                                        const double *__restrict__ x, KDev K,
                                                        int par) {
    const int nb = gridDim.x;
    double sx[NR] = {};
    if (A.u1) load_partials<NR>(K.partX, nb, sx);
    double acc5[5 * NR] = {};
    double *q = K.q[par];
    for (int64_t it = 0;; ++it) {
        const int64_t row = row_of(it);
        if (row - threadIdx.x >= A.n) break;
        if (row < A.n) {
            double acc[1][NR] = {};
            const double *ws[1] = {A.w};
            rbf::ell_row<KT, 1>(A.idx, ws, A.n, row, A.k, GatherN<NR>{x, A.n}, acc);
            const double u1 = A.u1 ? A.u1[row] * A.vscale : 0.0;
#pragma unroll
            for (int c = 0; c < NR; ++c) {
                const int64_t o = c * A.n + row;
                const double rr = b[o] - (acc[0][c] + u1 * sx[c]);
                double *qr = q + row * 4 * NR;
                qr[c] = rr;
                qr[NR + c] = 0.0;
                qr[2 * NR + c] = 0.0;
                qr[3 * NR + c] = 0.0;
                K.rh[o] = rr;
                acc5[0 * NR + c] += rr * rr;
                acc5[1 * NR + c] += rr * rr;
                acc5[2 * NR + c] += rr;
                acc5[3 * NR + c] += b[o] * b[o];
            }
        }
    }
    store_partials<5 * NR>(acc5, K.partA[par], nb);
    if (blockIdx.x == 0 && threadIdx.x < NR) {
        K.flag[threadIdx.x] = 0;
        K.iters[threadIdx.x] = 0;
    }
}

// On-the-fly D^-1 p' at a gathered column j (see k_kry_a).
template <int NR, bool JAC>
struct GatherP {
    static constexpr int NV = NR;
    const double *q, *dinv;
    double al[NR], om[NR], be[NR];
    __device__ __forceinline__ void operator()(int j, double (&out)[NR]) const {
        const double dj = JAC ? dinv[j] : 1.0;
        const double2 *qj = reinterpret_cast<const double2 *>(q + (int64_t)j * 4 * NR);
        double e[4 * NR];
#pragma unroll
        for (int h = 0; h < 2 * NR; ++h) {
            const double2 d = qj[h];
            e[2 * h] = d.x;
            e[2 * h + 1] = d.y;
        }
#pragma unroll
        for (int c = 0; c < NR; ++c) {
            const double rj = e[c], vj = e[NR + c], tj = e[2 * NR + c], pj = e[3 * NR + c];
            const double rn = (rj - al[c] * vj) - om[c] * tj;
            out[c] = dj * (rn + be[c] * (pj - om[c] * vj));
        }
    }
};

// On-the-fly D^-1 s at a gathered column j (see k_kry_b).
template <int NR, bool JAC>
struct GatherS {
    static constexpr int NV = NR;
    const double *q, *dinv;
    double al[NR];
    __device__ __forceinline__ void operator()(int j, double (&out)[NR]) const {
        const double dj = JAC ? dinv[j] : 1.0;
        const double2 *qj = reinterpret_cast<const double2 *>(q + (int64_t)j * 4 * NR);
        double e[2 * NR];
#pragma unroll
        for (int h = 0; h < NR; ++h) {
            const double2 d = qj[h];
            e[2 * h] = d.x;
            e[2 * h + 1] = d.y;
        }
#pragma unroll
        for (int c = 0; c < NR; ++c) out[c] = dj * (e[c] - al[c] * e[NR + c]);
    }
};

// Iteration i, first half.  par = i & 1: read buffers [par], write [par^1].
template <int NR, int KT, bool JAC>
__global__ void __launch_bounds__(kThreads) k_kry_a(EllM A, KDev K, double *__restrict__ x,
                                                     int i, int i0, int par) {
    if (all_done(K.flag, NR)) return;
    const int nb = gridDim.x;
    const bool first = (i == i0);
    double ra[5 * NR], rb[4 * NR];
    load_partials<5 * NR>(K.partA[par], nb, ra);
    if (!first) load_partials<4 * NR>(K.partB, nb, rb);
    GatherP<NR, JAC> g;
    g.q = K.q[par];
    g.dinv = A.dinv;
    double sp[NR];
    bool active[NR];
#pragma unroll
    for (int c = 0; c < NR; ++c) {
        active[c] = K.flag[c] == 0;
        double rho, om = 0.0, al = 0.0, be = 0.0;
        if (first) {
            rho = ra[0 * NR + c];
            sp[c] = ra[2 * NR + c];  // p' = r0
        } else {
            const double *pr = K.rec + ((int64_t)(i - 1) * NR + c) * 4;
            al = pr[1];
            om = (rb[1 * NR + c] != 0.0) ? rb[0 * NR + c] / rb[1 * NR + c] : 0.0;
            rho = -om * rb[2 * NR + c];
            be = (rho / pr[0]) * (al / om);
            // omega = 0 gives rho = 0, which the breakdown test of k_kry_b turns
            // into a restart; keep the direction finite meanwhile.
            if (!isfinite(be)) be = 0.0;
            // sum of p' from exact sums of r, p, v (this half) and t (k_kry_b)
            const double srn = ra[2 * NR + c] - al * ra[4 * NR + c] - om * rb[3 * NR + c];
            sp[c] = srn + be * (ra[3 * NR + c] - om * ra[4 * NR + c]);
        }
        g.al[c] = al;
        g.om[c] = om;
        g.be[c] = be;
        if (active[c] && blockIdx.x == 0 && threadIdx.x == 0) {
            K.rec[((int64_t)i * NR + c) * 4 + 0] = rho;
            if (first) {
                K.bb[c] = ra[3 * NR + c];
                K.rhrh[c] = ra[1 * NR + c];
            } else {
                K.rec[((int64_t)(i - 1) * NR + c) * 4 + 2] = om;
            }
        }
    }
    double *qout = K.q[par ^ 1];
    double acc5[5 * NR] = {};
    for (int64_t it = 0;; ++it) {
        const int64_t row = row_of(it);
        if (row - threadIdx.x >= A.n) break;
        if (row < A.n) {
            double acc[1][NR] = {};
            const double *ws[1] = {A.w};
            rbf::ell_row<KT, 1, decltype(g), (KT > 0 ? 7 : KT)>(A.idx, ws, A.n, row, A.k, g, acc);
            const double u1 = A.u1 ? A.u1[row] * A.vscale : 0.0;
            const double di = JAC ? A.dinv[row] : 1.0;
            const double *qi = g.q + row * 4 * NR;
            double *qo = qout + row * 4 * NR;
#pragma unroll
            for (int c = 0; c < NR; ++c) {
                if (!active[c]) continue;
                const int64_t o = c * A.n + row;
                const double vo = qi[NR + c], po = qi[3 * NR + c];
                const double s = qi[c] - g.al[c] * vo;
                const double rn = s - g.om[c] * qi[2 * NR + c];
                if (!first) x[o] = x[o] + g.al[c] * (di * po) + g.om[c] * (di * s);
                const double pn = rn + g.be[c] * (po - g.om[c] * vo);
                const double vn = acc[0][c] + u1 * sp[c];
                qo[c] = rn;
                qo[NR + c] = vn;
                qo[3 * NR + c] = pn;
                acc5[0 * NR + c] += K.rh[o] * vn;
                acc5[1 * NR + c] += rn * rn;
                acc5[2 * NR + c] += rn;
                acc5[3 * NR + c] += pn;
                acc5[4 * NR + c] += vn;
            }
        }
    }
    store_partials<5 * NR>(acc5, K.partA[par ^ 1], nb);
}

// Iteration i, second half: convergence test on ||r'||, alpha, t = A D^-1 s.
template <int NR, int KT, bool JAC>
__global__ void __launch_bounds__(kThreads) k_kry_b(EllM A, KDev K, int i, int par,
                                                     double tol2) {
    if (all_done(K.flag, NR)) return;
    const int nb = gridDim.x;
    double ra[5 * NR];
    load_partials<5 * NR>(K.partA[par ^ 1], nb, ra);
    GatherS<NR, JAC> g;
    g.q = K.q[par ^ 1];
    g.dinv = A.dinv;
    double ss[NR];
    bool active[NR];
    bool any = false;
#pragma unroll
    for (int c = 0; c < NR; ++c) {
        active[c] = K.flag[c] == 0;
        const double rho = K.rec[((int64_t)i * NR + c) * 4];
        const double rv = ra[0 * NR + c], rr = ra[1 * NR + c];
        const double al = rho / rv;
        g.al[c] = al;
        ss[c] = ra[2 * NR + c] - al * ra[4 * NR + c];
        if (!active[c]) continue;
        const double bb = K.bb[c], rhrh = K.rhrh[c];
        const bool bad = !isfinite(rr) || !isfinite(rho);
        const bool conv = !bad && (rr <= tol2 * fmax(bb, 1e-300) || rr == 0.0);
        const bool brk = !bad && !conv &&
                         (!(fabs(rho) > kBreakdown * sqrt(rr * rhrh)) || !isfinite(al));
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            double *rc = K.rec + ((int64_t)i * NR + c) * 4;
            rc[1] = al;
            rc[3] = rr;
            if (bad) K.flag[c] = -1;
            else if (conv) {
                K.flag[c] = 1;
                K.iters[c] = i;
            } else if (brk) {
                K.flag[c] = 2;
                K.iters[c] = i;
            }
        }
        if (bad || conv || brk) active[c] = false;
        else any = true;
    }
    if (!any) return;
    double acc4[4 * NR] = {};
    for (int64_t it = 0;; ++it) {
        const int64_t row = row_of(it);
        if (row - threadIdx.x >= A.n) break;
        if (row < A.n) {
            double acc[1][NR] = {};
            const double *ws[1] = {A.w};
            rbf::ell_row<KT, 1, decltype(g), (KT > 0 ? 7 : KT)>(A.idx, ws, A.n, row, A.k, g, acc);
            const double u1 = A.u1 ? A.u1[row] * A.vscale : 0.0;
            double *qr = K.q[par ^ 1] + row * 4 * NR;
#pragma unroll
            for (int c = 0; c < NR; ++c) {
                const int64_t o = c * A.n + row;
                const double tv = acc[0][c] + u1 * ss[c];
                const double s = qr[c] - g.al[c] * qr[NR + c];
                qr[2 * NR + c] = tv;
                acc4[0 * NR + c] += tv * s;
                acc4[1 * NR + c] += tv * tv;
                acc4[2 * NR + c] += K.rh[o] * tv;
                acc4[3 * NR + c] += tv;
            }
        }
    }
    store_partials<4 * NR>(acc4, K.partB, nb);
}

// True residual ||b - A x||^2 per right-hand side (for the statistics).
template <int NR, int KT>
__global__ void __launch_bounds__(kThreads) k_resid(EllM A, const double *__restrict__ b,
                                                     const double *__restrict__ x, double *part,
                                                     const double *partX) {
    double sx[NR] = {};
    if (A.u1) load_partials<NR>(partX, gridDim.x, sx);
    double acc2[NR] = {};
    for (int64_t it = 0;; ++it) {
        const int64_t r = row_of(it);
        if (r - threadIdx.x >= A.n) break;
        if (r < A.n) {
            double acc[1][NR] = {};
            const double *ws[1] = {A.w};
            rbf::ell_row<KT, 1>(A.idx, ws, A.n, r, A.k, GatherN<NR>{x, A.n}, acc);
            const double u1 = A.u1 ? A.u1[r] * A.vscale : 0.0;
#pragma unroll
            for (int c = 0; c < NR; ++c) {
                const double e = b[c * A.n + r] - (acc[0][c] + u1 * sx[c]);
                acc2[c] += e * e;
            }
        }
    }
    store_partials<NR>(acc2, part, gridDim.x);
}

// ------------------------------------------ lattice preconditioner --
// Right preconditioner of the pressure system when the P-nodes are a
// jittered (K+1) x (K+1) lattice (vertex (i, j) near (i h, j h), h = 1/K,
// row-major, boundary vertices on the walls):
//   P^-1 = J (L5 + chi c 1^T)^-1 D^-1
// D: the row scale of the stored Poisson rows; L5: the 5-point Laplacian of
// the unjittered lattice with one-sided Neumann rows (z_w - z_in) / |w - in|
// to the inward lattice neighbour (the diagonal one at corners); chi c 1^T:
// the same zero-mean border as the operator; J: bilinear interpolation from
// the lattice points to the actual node positions.  L5 is inverted exactly:
// the wall rows give z_w = z_in + |w - in| g_w, which leaves on the (K-1)^2
// interior nodes the separable operator (T (x) I + I (x) T) / h^2, T the
// 1-D second difference with Neumann ends.  The x-direction is
// diagonalised by the DCT-II basis Q (T = Q Lam Q^-1): a dense product
// Q^-1 X on the matrix cores (k_pc_gemm, FP64 MFMA); for each x-mode k the
// y-direction system (T + lam_k I) w = h^2 t is tridiagonal and is solved by
// one wavefront per mode (k_pc_tri: elimination inside per-lane chunks, then
// cyclic reduction across the lanes); the product Q W returns to the
// lattice.  Mode k = 0 is
// singular: its right-hand side loses its mean (recorded: it fixes the
// constant through the border), the last unknown is fixed and the solution
// shifted to zero mean.
//
// Interior arrays, n = K - 1, X(a, b) / Z(a, b) belong to lattice node
// (i, j) = (a + 1, b + 1):
//   X  reduced right-hand side, row-major  (a n + b); then Z, column-major
//   T  Q^-1 X, row-major (k n + b)
//   W  tridiagonal solutions, row-major (k n + b)
// The constant shift needs the lattice sum of the boundary values:
// sum_w Z(in(w)) = sum_kb W(k, b) V(k, b) with V = Q^T w (w counts the
// boundary nodes clamped to each interior node), reduced per block by
// k_pc_tri per mode, plus sum_w |w - in(w)| g_w, reduced by the kernel that
// builds X.
// The transform arrays are FP64, or FP32 when f32 is set (mixed precision:
// the preconditioner only shapes the iteration, the residuals stay FP64).
struct Lat {
    int K, n, ntiles, f32;
    double h, c;           // spacing; border scale
    const double *rs;      // [M] row scale of the stored Poisson rows
    const int *cell;       // [M] lower-left lattice node of the cell holding the node
    const double *fx, *fy; // [M] bilinear coordinates in that cell
    const void *Q, *Qi;    // [n * n] column-major
    const double *lam;     // [n] eigenvalues of T (unit spacing)
    const double *V;       // [n * n] boundary weights in (k, b), at k n + b
    void *X, *T, *W;       // [n * n] work (Z overwrites X)
    double *mean;          // [1] zero-mode coefficient (mean of the reduced rhs)
    double *partW;         // [n] per-mode sums of W o V
    const int *flag;       // iteration flag: the stages exit once it is set
};

__device__ __forceinline__ void lat_store(const Lat &L, void *a, int64_t e, double v) {
    if (L.f32) static_cast<float *>(a)[e] = (float)v;
    else static_cast<double *>(a)[e] = v;
}
__device__ __forceinline__ double lat_load(const Lat &L, const void *a, int64_t e) {
    return L.f32 ? (double)static_cast<const float *>(a)[e] : static_cast<const double *>(a)[e];
}

// Preconditioned BiCGSTAB vectors and scalars (one right-hand side).
// p is double-buffered by iteration parity (the kernel that rewrites it also
// recomputes the new value at wall neighbours from the old one).
struct PKry {
    double *r, *rh, *p[2], *v, *s, *t, *ph, *sh;
    double *partI;  // init: {rho_0, ||b||^2}
    double *part1;  // k_pc_dir: ||r||^2, boundary sum of the reduced rhs of p
    double *partGs; // k_pc_s: boundary sum of the reduced rhs of s
    double *part3;  // k_pc_av (v): (rh, v)
    double *part6;  // k_pc_av (t): (t, s), (t, t), (rh, t)
    double *partS;  // k_pc_post: sum of the preconditioned vector
    double *rec;    // per iteration {rho, alpha, omega, ||r||^2}
    double *bb, *rhrh;
    double *best;   // [2][2] {best ||r||^2, its iteration}, by iteration parity
    // Status block read by the host after each batch in one copy: flag,
    // iters, then (as doubles) ||r_i||^2 of the last tested iteration i, of
    // iteration max(i0, i - 4), and ||b||^2.
    int *flag, *iters;
    double *stat;
};

// Iterations without progress after which the preconditioned iteration
// restarts; the window doubles after every restart of a solve.
constexpr int kStall = 8;

// Reduced right-hand side at interior lattice node `row` = (i, j), from the
// values val(node) of the vector y being preconditioned: D^-1 y with the
// wall values moved to the right-hand side.  At a boundary node, returns
// its term |w - in(w)| (D^-1 y)_w of the boundary sum (0 elsewhere).
// rself = L.rs[row], loaded by the caller.
template <class V>
__device__ __forceinline__ double pc_reduce(const Lat &L, int64_t row, double vself, double rself,
                                            V val) {
    const int K = L.K, K1 = K + 1;
    const int i = (int)(row % K1), j = (int)(row / K1);
    const bool bi = (i == 0 || i == K), bj = (j == 0 || j == K);
    if (bi || bj) return ((bi && bj) ? L.h * 1.4142135623730951 : L.h) * (vself / rself);
    double g = vself / rself;
    double wsum = 0.0;
    if (i == 1) wsum += val(row - 1) / L.rs[row - 1];
    if (i == K - 1) wsum += val(row + 1) / L.rs[row + 1];
    if (j == 1) wsum += val(row - K1) / L.rs[row - K1];
    if (j == K - 1) wsum += val(row + K1) / L.rs[row + K1];
    g -= wsum / L.h;
    lat_store(L, L.X, (int64_t)(i - 1) * L.n + (j - 1), g);
    return 0.0;
}

// r0 = b - A x, rh = r0.
template <int KT>
__global__ void __launch_bounds__(kThreads) k_pc_init(EllM A, const double *__restrict__ b,
                                                       const double *__restrict__ x, PKry K,
                                                       const double *partX) {
    const int nb = gridDim.x;
    double sx[1] = {0.0};
    if (A.u1) load_partials<1>(partX, nb, sx);
    double acc[2] = {};
    for (int64_t it = 0;; ++it) {
        const int64_t row = row_of(it);
        if (row - threadIdx.x >= A.n) break;
        if (row < A.n) {
            double ax[1][1] = {};
            const double *ws[1] = {A.w};
            rbf::ell_row<KT, 1>(A.idx, ws, A.n, row, A.k, GatherN<1>{x, A.n}, ax);
            const double u1 = A.u1 ? A.u1[row] * A.vscale : 0.0;
            const double rr = b[row] - (ax[0][0] + u1 * sx[0]);
            K.r[row] = rr;
            K.rh[row] = rr;
            acc[0] += rr * rr;
            acc[1] += b[row] * b[row];
        }
    }
    store_partials<2>(acc, K.partI, nb);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        K.flag[0] = 0;
        K.iters[0] = 0;
    }
}

// Iteration i, step 1: finish iteration i-1 (r = s - omega t,
// x += alpha ph + omega sh), new direction p = r + beta (p - omega v), and
// the reduced right-hand side of p for the preconditioner.  Breakdowns are
// detected by k_pc_s from the recorded scalars, so that every block of this
// kernel performs the same update.
__global__ void __launch_bounds__(kThreads) k_pc_dir(PKry K, Lat L, double *__restrict__ x,
                                                      int64_t m, int i, int i0) {
    const int nb = gridDim.x;
    const bool first = (i == i0);
    const int par = i & 1;
    const double *pold = K.p[par ^ 1];
    double *pnew = K.p[par];
    // Every load that does not depend on another goes out before the first
    // wait: the flag, the partial sums, the recorded scalars and the vectors
    // of this thread's first row.
    const int fl = K.flag[0];
    double q[3] = {0.0, 0.0, 0.0};
    if (first) {
        for (int b = threadIdx.x; b < nb; b += blockDim.x) {
            q[0] += K.partI[b];
            q[1] += K.partI[nb + b];
        }
    } else {
        for (int b = threadIdx.x; b < nb; b += blockDim.x) {
            q[0] += K.part6[b];
            q[1] += K.part6[nb + b];
            q[2] += K.part6[2 * nb + b];
        }
    }
    const double pr0 = first ? 0.0 : K.rec[(int64_t)(i - 1) * 4 + 0];
    const double pr1 = first ? 0.0 : K.rec[(int64_t)(i - 1) * 4 + 1];
    const int64_t row0 = row_of(0);
    double f_r = 0.0, f_s = 0.0, f_t = 0.0, f_po = 0.0, f_v = 0.0, f_ph = 0.0, f_sh = 0.0,
           f_x = 0.0, f_rs = 1.0;
    if (row0 < m) {
        f_rs = L.rs[row0];
        if (first) {
            f_r = K.r[row0];
        } else {
            f_s = K.s[row0];
            f_t = K.t[row0];
            f_po = pold[row0];
            f_v = K.v[row0];
            f_ph = K.ph[row0];
            f_sh = K.sh[row0];
            f_x = x[row0];
        }
    }
    if (fl != 0) return;
    {
        __shared__ double lds[3 * (kThreads / 64)];
        rbf::block_sum<3>(q, lds);
    }
    double al = 0.0, om = 0.0, be = 0.0, rho;
    if (first) {
        rho = q[0];
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            K.bb[0] = q[1];
            K.rhrh[0] = q[0];
            K.rec[(int64_t)i * 4 + 0] = rho;
        }
    } else {
        al = pr1;
        om = (q[1] != 0.0) ? q[0] / q[1] : 0.0;
        rho = -om * q[2];  // (rh, s) = 0 by the choice of alpha
        be = (rho / pr0) * (al / om);
        if (!isfinite(be)) be = 0.0;  // omega = 0: rho = 0, restarted by k_pc_s
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            K.rec[(int64_t)(i - 1) * 4 + 2] = om;
            K.rec[(int64_t)i * 4 + 0] = rho;
        }
    }
    auto pval = [&](int64_t j) {
        if (first) return K.r[j];
        const double rn = K.s[j] - om * K.t[j];
        return rn + be * (pold[j] - om * K.v[j]);
    };
    double acc[2] = {0.0, 0.0};
    for (int64_t it = 0;; ++it) {
        const int64_t row = row_of(it);
        if (row - threadIdx.x >= m) break;
        if (row < m) {
            const bool pre = (it == 0);
            double rn, pn;
            if (first) {
                rn = pre ? f_r : K.r[row];
                pn = rn;
            } else {
                const double sv = pre ? f_s : K.s[row], tv = pre ? f_t : K.t[row];
                const double pv = pre ? f_po : pold[row], vv = pre ? f_v : K.v[row];
                const double phv = pre ? f_ph : K.ph[row], shv = pre ? f_sh : K.sh[row];
                const double xv = pre ? f_x : x[row];
                rn = sv - om * tv;
                x[row] = xv + al * phv + om * shv;
                K.r[row] = rn;
                pn = rn + be * (pv - om * vv);
            }
            pnew[row] = pn;
            acc[0] += rn * rn;
            acc[1] += pc_reduce(L, row, pn, pre ? f_rs : L.rs[row], pval);
        }
    }
    store_partials<2>(acc, K.part1, nb);
}

// Iteration i, step 2: convergence test on ||r_i||, alpha = rho / (rh, v),
// s = r - alpha v and its reduced right-hand side.
__global__ void __launch_bounds__(kThreads) k_pc_s(PKry K, Lat L, int64_t m, int i, int i0,
                                                    double tol2, int win) {
    const int nb = gridDim.x;
    // Loads first (see k_pc_dir).
    const int fl = K.flag[0];
    double q[2] = {0.0, 0.0};
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
        q[0] += K.part1[b];
        q[1] += K.part3[b];
    }
    const double rho = K.rec[(int64_t)i * 4];
    const double bb = K.bb[0], rhrh = K.rhrh[0];
    // Stagnation: no 0.1% decrease of the best ||r||^2 for win iterations
    // is handled like a breakdown (restart from the true residual).  The best
    // value is double-buffered by parity: read from the previous launch,
    // written for the next one.
    const double *bprev = K.best + ((i + 1) & 1) * 2;
    const double bp0 = bprev[0], bp1 = bprev[1];
    const int64_t row0 = row_of(0);
    double f_r = 0.0, f_v = 0.0, f_rs = 1.0;
    if (row0 < m) {
        f_r = K.r[row0];
        f_v = K.v[row0];
        f_rs = L.rs[row0];
    }
    if (fl != 0) return;
    {
        __shared__ double lds[2 * (kThreads / 64)];
        rbf::block_sum<2>(q, lds);
    }
    const double rr = q[0], rv = q[1];
    const double al = rho / rv;
    const bool bad = !isfinite(rr) || !isfinite(rho);
    const bool conv = !bad && (rr <= tol2 * fmax(bb, 1e-300) || rr == 0.0);
    const bool fresh = (i == i0);
    const double best = fresh ? rr : bp0;
    const int best_it = fresh ? i : (int)bp1;
    const bool better = fresh || rr < 0.999 * best;
    const bool stall = !better && (i - best_it >= win);
    const bool brk = !bad && !conv &&
                     (!(fabs(rho) > kBreakdown * sqrt(rr * rhrh)) || !isfinite(al) || stall);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        double *rc = K.rec + (int64_t)i * 4;
        rc[1] = al;
        rc[3] = rr;
        double *bnext = K.best + (i & 1) * 2;
        bnext[0] = better ? rr : best;
        bnext[1] = better ? (double)i : (double)best_it;
        const int back = max(i0, i - 4);
        K.stat[0] = rr;
        K.stat[1] = (back == i) ? rr : K.rec[(int64_t)back * 4 + 3];
        K.stat[2] = bb;
        if (bad) K.flag[0] = -1;
        else if (conv || brk) {
            K.flag[0] = conv ? 1 : 2;
            K.iters[0] = i;
        }
    }
    if (bad || conv || brk) return;
    auto sval = [&](int64_t j) { return K.r[j] - al * K.v[j]; };
    double acc[1] = {0.0};
    for (int64_t it = 0;; ++it) {
        const int64_t row = row_of(it);
        if (row - threadIdx.x >= m) break;
        if (row < m) {
            const bool pre = (it == 0);
            const double sv = (pre ? f_r : K.r[row]) - al * (pre ? f_v : K.v[row]);
            K.s[row] = sv;
            acc[0] += pc_reduce(L, row, sv, pre ? f_rs : L.rs[row], sval);
        }
    }
    store_partials<1>(acc, K.partGs, nb);
}

// Reduced right-hand side of an explicit vector y (rbf_solver_apply_precond).
__global__ void __launch_bounds__(kThreads) k_pc_pre(Lat L, const double *__restrict__ y, int64_t m,
                                                      double *partG) {
    auto yval = [&](int64_t j) { return y[j]; };
    double acc[1] = {0.0};
    for (int64_t it = 0;; ++it) {
        const int64_t row = row_of(it);
        if (row - threadIdx.x >= m) break;
        if (row < m) acc[0] += pc_reduce(L, row, y[row], L.rs[row], yval);
    }
    store_partials<1>(acc, partG, gridDim.x);
}

// The two transforms of the interior solve, one 16x16 tile per workgroup of
// kGemmWaves waves.  STAGE 0: T = Q^-1 X; STAGE 1: Z = Q W (into X).
// Split-K factor and chunk: with n <= 4 kGemmWaves kGemmChunk (K <= 449)
// a wave's whole k-share is loaded before its MFMAs (ONESHOT).
constexpr int kGemmWaves = 8;
constexpr int kGemmChunk = 14;
template <int STAGE, bool ONESHOT, class TP>
__global__ void __launch_bounds__(64 * kGemmWaves) k_pc_gemm(Lat L) {
    // The flag is tested first: a launch after convergence would otherwise
    // fetch its whole operand share before exiting.
    if (*L.flag != 0) return;
    const int n = L.n, nt = (n + 15) / 16;
    const int ti = (int)(blockIdx.x % nt), tj = (int)(blockIdx.x / nt);
    const TP *A = static_cast<const TP *>(STAGE == 0 ? L.Qi : L.Q);
    const TP *B = static_cast<const TP *>(STAGE == 0 ? L.X : L.W);
    TP *C = static_cast<TP *>(STAGE == 0 ? L.T : L.X);
    // T row-major (one mode per row, read whole by k_pc_tri), Z column-major.
    rbf::mfma_block<TP, 1, 1, kGemmWaves, kGemmChunk, ONESHOT>(
        n, A, B, ti, tj, [&](int i, int j, TP v) {
            if constexpr (STAGE == 0) C[(int64_t)i * n + j] = v;
            else C[i + (int64_t)j * n] = v;
        });
}

// For each x-mode k (one wavefront): (T + lam_k I) w = h^2 t along y.  The
// rows are split into nch <= 64 chunks of 2-8 consecutive rows, one per
// lane.  Each lane eliminates inside its chunk
// (a downward and an upward sweep that leave every row coupled only to the
// chunk's first and last unknowns), the first and last rows of all chunks
// reduce to a tridiagonal system in the chunks' first unknowns, one per
// lane, solved by cyclic reduction across the wavefront (shuffles), and each
// lane recovers its rows.  The systems are diagonally dominant, so no
// pivoting.  Mode 0 is singular: its right-hand side loses its mean
// (recorded in *L.mean), its last row is dropped (w_{n-1} = 0) and the
// solution is shifted to zero mean.  Writes W row-major and the sum of
// W o V over the mode into partW[k].
constexpr int kTriChunk = 8;  // rows per lane: n <= 64 kTriChunk (K <= 513)
template <class TP>
__global__ void __launch_bounds__(64) k_pc_tri(Lat L) {
    __shared__ double sz[64 * kTriChunk];
    const int n = L.n, k = blockIdx.x, lane = threadIdx.x;
    const TP *T = static_cast<const TP *>(L.T);
    // Every global load of the kernel is issued before the flag test, so
    // that the whole kernel waits on one memory round trip.
    double tv[kTriChunk], vv[kTriChunk];
#pragma unroll
    for (int m = 0; m < kTriChunk; ++m) {
        const int i = lane + 64 * m;
        tv[m] = (i < n) ? (double)T[(int64_t)k * n + i] : 0.0;
        vv[m] = (i < n) ? L.V[(int64_t)k * n + i] : 0.0;
    }
    const double lamk = L.lam[k];
    if (*L.flag != 0) return;
    double tsum = 0.0;
#pragma unroll
    for (int m = 0; m < kTriChunk; ++m) {
        const int i = lane + 64 * m;
        if (i < n) sz[i] = tv[m];
        tsum += tv[m];
    }
    const int size = (k == 0) ? n - 1 : n;
    double shift = 0.0;
    if (k == 0) {  // block-uniform branch
        shift = rbf::wave_sum(tsum) / n;
        if (lane == 0) *L.mean = shift;
    }
    __syncthreads();
    const double h2 = L.h * L.h;
    const int nch = min(64, max(1, size / 2));
    const int base = size > 0 ? size / nch : 0, extra = size > 0 ? size % nch : 0;
    const bool act = lane < nch && size > 0;
    const int len = act ? base + (lane < extra ? 1 : 0) : 0;
    const int r0 = lane * base + min(lane, extra);
    auto row = [&](int i, double &a, double &b, double &c, double &d) {
        a = (i == 0) ? 0.0 : 1.0;
        c = (i == size - 1) ? 0.0 : 1.0;
        b = ((i == 0 || i == n - 1) ? -1.0 : -2.0) + lamk;
        d = h2 * (sz[i] - shift);
    };
    // Downward sweep: row j >= 1 becomes ap_j x_first + x_j + cp_j x_{j+1} = dp_j
    // (row 0 normalised: ap_0 couples to the previous chunk's last unknown).
    double ap[kTriChunk], cp[kTriChunk], dp[kTriChunk];
    double fa = 0.0, fc = 0.0, fd = 0.0;  // last row: fa x_first + x_last + fc x_next = fd
#pragma unroll
    for (int j = 0; j < kTriChunk; ++j) {
        ap[j] = cp[j] = dp[j] = 0.0;
        if (j < len) {
            double a, b, c, d;
            row(r0 + j, a, b, c, d);
            if (j < 2) {
                const double r = 1.0 / b;
                ap[j] = a * r;
                cp[j] = c * r;
                dp[j] = d * r;
            } else {
                const double r = 1.0 / (b - a * cp[j - 1]);
                ap[j] = -a * ap[j - 1] * r;
                cp[j] = c * r;
                dp[j] = (d - a * dp[j - 1]) * r;
            }
            if (j == len - 1) {
                fa = ap[j];
                fc = cp[j];
                fd = dp[j];
            }
        }
    }
    // Upward sweep: rows 1..len-2 become ap_j x_first + x_j + cp_j x_last = dp_j.
#pragma unroll
    for (int j = kTriChunk - 3; j >= 1; --j) {
        if (j <= len - 3) {
            ap[j] -= cp[j] * ap[j + 1];
            dp[j] -= cp[j] * dp[j + 1];
            cp[j] = -cp[j] * cp[j + 1];
        }
    }
    // First row: ea x_prev_last + eb x_first + ec x_last = ed.
    double ea = ap[0], eb = 1.0, ec = cp[0], ed = dp[0];
    if (len >= 3) {
        eb = 1.0 - cp[0] * ap[1];
        ec = -cp[0] * cp[1];
        ed = dp[0] - cp[0] * dp[1];
    }
    // Eliminate the last unknowns (x_last = fd - fa x_first - fc x_next_first):
    // A x_prev_first + B x_first + C x_next_first = D, one row per lane.
    const double fa_m = __shfl(fa, lane > 0 ? lane - 1 : 0, 64);
    const double fc_m = __shfl(fc, lane > 0 ? lane - 1 : 0, 64);
    const double fd_m = __shfl(fd, lane > 0 ? lane - 1 : 0, 64);
    double A = 0.0, B = 1.0, C = 0.0, D = 0.0;
    if (len == 1) {  // size == 1: a single unknown
        B = eb;
        D = ed;
    } else if (act) {
        const double em = (lane > 0) ? ea : 0.0;
        A = -em * fa_m;
        B = eb - em * fc_m - ec * fa;
        C = -ec * fc;
        D = ed - em * fd_m - ec * fd;
    }
    for (int st = 1; st < 64; st <<= 1) {
        const bool lo = lane >= st, hi = lane + st < 64;
        const int sl = lo ? lane - st : lane, sh = hi ? lane + st : lane;
        const double am = __shfl(A, sl, 64), bm = __shfl(B, sl, 64), cm = __shfl(C, sl, 64),
                     dm = __shfl(D, sl, 64);
        const double aq = __shfl(A, sh, 64), bq = __shfl(B, sh, 64), cq = __shfl(C, sh, 64),
                     dq = __shfl(D, sh, 64);
        const double al = lo ? -A / bm : 0.0, ga = hi ? -C / bq : 0.0;
        const double A2 = lo ? al * am : 0.0, C2 = hi ? ga * cq : 0.0;
        const double B2 = B + (lo ? al * cm : 0.0) + (hi ? ga * aq : 0.0);
        const double D2 = D + (lo ? al * dm : 0.0) + (hi ? ga * dq : 0.0);
        A = A2;
        B = B2;
        C = C2;
        D = D2;
    }
    const double x0 = D / B;
    const double xn = __shfl(x0, lane < 63 ? lane + 1 : lane, 64);
    const double xl = fd - fa * x0 - fc * xn;
    __syncthreads();
    if (k == 0 && lane == 0) sz[n - 1] = 0.0;  // the dropped last unknown of mode 0
#pragma unroll
    for (int j = 0; j < kTriChunk; ++j) {
        if (j < len) {
            const double z = (j == 0) ? x0 : (j == len - 1) ? xl : dp[j] - ap[j] * x0 - cp[j] * xl;
            sz[r0 + j] = z;
        }
    }
    __syncthreads();
    double zmean = 0.0;
    if (k == 0) {
        double s = 0.0;
        for (int i = lane; i < n; i += 64) s += sz[i];
        zmean = rbf::wave_sum(s) / n;
    }
    double acc = 0.0;
#pragma unroll
    for (int m = 0; m < kTriChunk; ++m) {
        const int i = lane + 64 * m;
        if (i < n) {
            const double z = sz[i] - zmean;
            static_cast<TP *>(L.W)[(int64_t)k * n + i] = (TP)z;
            acc += z * vv[m];
        }
    }
    acc = rbf::wave_sum(acc);
    if (lane == 0) L.partW[k] = acc;
}

// Lattice value of L5^-1 at node (i, j), before the constant shift (Z in X).
__device__ __forceinline__ double pc_lattice(const Lat &L, const double *y, int i, int j) {
    const int K = L.K;
    const int ci = min(max(i, 1), K - 1), cj = min(max(j, 1), K - 1);
    double z = lat_load(L, L.X, (int64_t)(ci - 1) + (int64_t)(cj - 1) * L.n);
    const bool bi = (i == 0 || i == K), bj = (j == 0 || j == K);
    if (bi || bj) {
        const int64_t node = (int64_t)j * (K + 1) + i;
        const double dist = (bi && bj) ? L.h * 1.4142135623730951 : L.h;
        z += dist * (y[node] / L.rs[node]);
    }
    return z;
}

// out = J (zl + alpha) at every node; alpha makes the lattice sum equal to
// the value the border prescribes (mean / c): the interior part of the
// lattice solution has zero sum (no zero mode), the boundary part is
// reduced from the partials of k_pc_tri (partW) and of the kernel that
// built X (partG, nbG blocks).  Writes block partials of sum(out).
__global__ void __launch_bounds__(kThreads) k_pc_post(Lat L, PKry K, const double *__restrict__ y,
                                                       double *__restrict__ out, int64_t m,
                                                       double *partS, const double *partG,
                                                       int nbG) {
    const int Kl = L.K;
    // The first row's cell data and the partial sums are loaded before the
    // flag test (one memory round trip for all of them).
    const int64_t row0 = row_of(0);
    int c_0 = 0;
    double fx_0 = 0.0, fy_0 = 0.0;
    if (row0 < m) {
        c_0 = L.cell[row0];
        fx_0 = L.fx[row0];
        fy_0 = L.fy[row0];
    }
    double bwg[2] = {0.0, 0.0};
    for (int b = threadIdx.x; b < L.n; b += blockDim.x) bwg[0] += L.partW[b];
    for (int b = threadIdx.x; b < nbG; b += blockDim.x) bwg[1] += partG[b];
    const double mean = *L.mean;
    if (K.flag[0] != 0) return;
    {
        __shared__ double lds[2 * (kThreads / 64)];
        rbf::block_sum<2>(bwg, lds);
    }
    const double alpha = (mean / L.c - (bwg[0] + bwg[1])) / (double)m;
    double acc[1] = {0.0};
    for (int64_t it = 0;; ++it) {
        const int64_t row = row_of(it);
        if (row - threadIdx.x >= m) break;
        if (row < m) {
            const int c = (it == 0) ? c_0 : L.cell[row];
            const int i0 = c % (Kl + 1), j0 = c / (Kl + 1);
            const double fx = (it == 0) ? fx_0 : L.fx[row], fy = (it == 0) ? fy_0 : L.fy[row];
            const double z00 = pc_lattice(L, y, i0, j0), z10 = pc_lattice(L, y, i0 + 1, j0);
            const double z01 = pc_lattice(L, y, i0, j0 + 1), z11 = pc_lattice(L, y, i0 + 1, j0 + 1);
            const double z = ((1.0 - fy) * ((1.0 - fx) * z00 + fx * z10) +
                              fy * ((1.0 - fx) * z01 + fx * z11)) + alpha;
            out[row] = z;
            acc[0] += z;
        }
    }
    store_partials<1>(acc, partS, gridDim.x);
}

// out = A y (+ rank-one border); MODE 0: partials (rh, out) -> part3,
// MODE 1: partials (out, s), (out, out), (rh, out) -> part6.
template <int KT, int MODE>
__global__ void __launch_bounds__(kThreads) k_pc_av(EllM A, PKry K, const double *__restrict__ y,
                                                     double *__restrict__ out) {
    const int nb = gridDim.x;
    // The flag and the partial sums of the border term are loaded together
    // and tested before the row's loads (a launch after convergence then
    // exits after one short round trip); the first row's indices and
    // vector entries go out before the partial sums are reduced.
    const int fl = K.flag[0];
    double sy[1] = {0.0};
    if (A.u1)
        for (int b = threadIdx.x; b < nb; b += blockDim.x) sy[0] += K.partS[b];
    auto rowval = [&](int64_t row, double &ay, double &u1, double &rh, double &sv) {
        rh = K.rh[row];
        sv = (MODE == 1) ? K.s[row] : 0.0;
        u1 = A.u1 ? A.u1[row] * A.vscale : 0.0;
        double a[1][1] = {};
        const double *ws[1] = {A.w};
        rbf::ell_row<KT, 1>(A.idx, ws, A.n, row, A.k, GatherN<1>{y, A.n}, a);
        ay = a[0][0];
    };
    if (fl != 0) return;
    const int64_t row0 = row_of(0);
    const bool has0 = row0 < A.n;
    constexpr int KP = KT > 0 ? KT : 1;
    int jj[KP];
    double f_u1 = 0.0, f_rh = 0.0, f_s = 0.0;
    if (KT > 0 && has0) {
#pragma unroll
        for (int q = 0; q < KP; ++q) jj[q] = rbf::ld_stream(A.idx + (int64_t)q * A.n + row0);
        f_rh = K.rh[row0];
        f_s = (MODE == 1) ? K.s[row0] : 0.0;
        f_u1 = A.u1 ? A.u1[row0] * A.vscale : 0.0;
    }
    if (A.u1) {
        __shared__ double lds[kThreads / 64];
        rbf::block_sum<1>(sy, lds);
    }
    constexpr int NQ = MODE == 0 ? 1 : 3;
    double acc[NQ] = {};
    for (int64_t it = 0;; ++it) {
        const int64_t row = row_of(it);
        if (row - threadIdx.x >= A.n) break;
        if (row < A.n) {
            double ay = 0.0, u1, rh, sv;
            if (KT > 0 && it == 0) {
                double ww[KP];
#pragma unroll
                for (int q = 0; q < KP; ++q) ww[q] = rbf::ld_stream(A.w + (int64_t)q * A.n + row0);
#pragma unroll
                for (int q = 0; q < KP; ++q) ay = fma(ww[q], y[jj[q]], ay);
                u1 = f_u1;
                rh = f_rh;
                sv = f_s;
            } else {
                rowval(row, ay, u1, rh, sv);
            }
            const double val = ay + u1 * sy[0];
            out[row] = val;
            if constexpr (MODE == 0) {
                acc[0] += rh * val;
            } else {
                acc[0] += val * sv;
                acc[1] += val * val;
                acc[2] += rh * val;
            }
        }
    }
    store_partials<NQ>(acc, MODE == 0 ? K.part3 : K.part6, nb);
}

// ------------------------------------ viscous solve, explicit vectors --
// Jacobi right-preconditioned BiCGSTAB for the two velocity components at
// once (stacked [2][N] vectors): the preconditioned directions p^ = D^-1 p
// and s^ = D^-1 s are written out, so the two products per iteration
// gather 16 bytes per neighbour.  Same scalar recurrences, flags and
// deterministic reductions as the pressure iteration, per component.
constexpr int kHR = 2;
struct HKry {
    double *r, *rh, *p[2], *v, *s, *t, *ph, *sh;  // [2][N] each
    double *partI;  // init: {rho_0 (2), ||b||^2 (2)}
    double *part1;  // ||r||^2 (2)
    double *part3;  // (rh, v) (2)
    double *part6;  // (t, s), (t, t), (rh, t) (2 each)
    double *rec;    // [iteration][component] {rho, alpha, omega, ||r||^2}
    double *bb, *rhrh;
    double *best;   // [parity][component][2] {best ||r||^2, its iteration}
    int *flag, *iters;
};

__device__ __forceinline__ bool h_done(const int *flag) { return flag[0] != 0 && flag[1] != 0; }

template <int KT>
__global__ void __launch_bounds__(kThreads) k_h_init(EllM A, const double *__restrict__ b,
                                                      const double *__restrict__ x, HKry K) {
    const int nb = gridDim.x;
    double acc[2 * kHR] = {};
    for (int64_t it = 0;; ++it) {
        const int64_t row = row_of(it);
        if (row - threadIdx.x >= A.n) break;
        if (row < A.n) {
            double ax[1][kHR] = {};
            const double *ws[1] = {A.w};
            rbf::ell_row<KT, 1>(A.idx, ws, A.n, row, A.k, GatherN<kHR>{x, A.n}, ax);
#pragma unroll
            for (int c = 0; c < kHR; ++c) {
                const int64_t o = c * A.n + row;
                const double rr = b[o] - ax[0][c];
                K.r[o] = rr;
                K.rh[o] = rr;
                acc[c] += rr * rr;
                acc[kHR + c] += b[o] * b[o];
            }
        }
    }
    store_partials<2 * kHR>(acc, K.partI, nb);
    if (blockIdx.x == 0 && threadIdx.x < kHR) {
        K.flag[threadIdx.x] = 0;
        K.iters[threadIdx.x] = 0;
    }
}

// Finish iteration i-1 and build the new direction (see k_pc_dir).
__global__ void __launch_bounds__(kThreads) k_h_dir(HKry K, const double *__restrict__ dinv,
                                                     double *__restrict__ x, int64_t n, int i, int i0) {
    if (h_done(K.flag)) return;
    const int nb = gridDim.x;
    const bool first = (i == i0);
    const int par = i & 1;
    double al[kHR] = {}, om[kHR] = {}, be[kHR] = {};
    bool act[kHR];
    double q[4 * kHR];
    if (first) load_partials<2 * kHR>(K.partI, nb, *reinterpret_cast<double(*)[2 * kHR]>(q));
    else load_partials<3 * kHR>(K.part6, nb, *reinterpret_cast<double(*)[3 * kHR]>(q));
#pragma unroll
    for (int c = 0; c < kHR; ++c) {
        act[c] = K.flag[c] == 0;
        double rho;
        if (first) {
            rho = q[c];
            if (blockIdx.x == 0 && threadIdx.x == 0) {
                K.bb[c] = q[kHR + c];
                K.rhrh[c] = q[c];
                K.rec[((int64_t)i * kHR + c) * 4] = rho;
            }
        } else {
            const double *pr = K.rec + ((int64_t)(i - 1) * kHR + c) * 4;
            al[c] = pr[1];
            const double ts = q[c], tt = q[kHR + c], rt = q[2 * kHR + c];
            om[c] = (tt != 0.0) ? ts / tt : 0.0;
            rho = -om[c] * rt;
            be[c] = (rho / pr[0]) * (al[c] / om[c]);
            if (!isfinite(be[c])) be[c] = 0.0;  // omega = 0: rho = 0, restarted by k_h_s
            if (blockIdx.x == 0 && threadIdx.x == 0 && act[c]) {
                K.rec[((int64_t)(i - 1) * kHR + c) * 4 + 2] = om[c];
                K.rec[((int64_t)i * kHR + c) * 4] = rho;
            }
        }
    }
    const double *pold = K.p[par ^ 1];
    double *pnew = K.p[par];
    double acc[kHR] = {};
    for (int64_t it = 0;; ++it) {
        const int64_t row = row_of(it);
        if (row - threadIdx.x >= n) break;
        if (row < n) {
            const double di = dinv[row];
#pragma unroll
            for (int c = 0; c < kHR; ++c) {
                if (!act[c]) continue;
                const int64_t o = c * n + row;
                double rn, pn;
                if (first) {
                    rn = K.r[o];
                    pn = rn;
                } else {
                    rn = K.s[o] - om[c] * K.t[o];
                    x[o] = x[o] + al[c] * K.ph[o] + om[c] * K.sh[o];
                    K.r[o] = rn;
                    pn = rn + be[c] * (pold[o] - om[c] * K.v[o]);
                }
                pnew[o] = pn;
                K.ph[o] = di * pn;
                acc[c] += rn * rn;
            }
        }
    }
    store_partials<kHR>(acc, K.part1, nb);
}

// out = A y for both components; MODE 0: partials (rh, out) -> part3;
// MODE 1: (out, s), (out, out), (rh, out) -> part6.
template <int KT, int MODE>
__global__ void __launch_bounds__(kThreads) k_h_av(EllM A, HKry K, const double *__restrict__ y,
                                                    double *__restrict__ out) {
    if (h_done(K.flag)) return;
    const int nb = gridDim.x;
    constexpr int NQ = (MODE == 0 ? 1 : 3) * kHR;
    double acc[NQ] = {};
    for (int64_t it = 0;; ++it) {
        const int64_t row = row_of(it);
        if (row - threadIdx.x >= A.n) break;
        if (row < A.n) {
            double ay[1][kHR] = {};
            const double *ws[1] = {A.w};
            rbf::ell_row<KT, 1>(A.idx, ws, A.n, row, A.k, GatherN<kHR>{y, A.n}, ay);
#pragma unroll
            for (int c = 0; c < kHR; ++c) {
                const int64_t o = c * A.n + row;
                const double val = ay[0][c];
                out[o] = val;
                const double rh = K.rh[o];
                if constexpr (MODE == 0) {
                    acc[c] += rh * val;
                } else {
                    const double sv = K.s[o];
                    acc[c] += val * sv;
                    acc[kHR + c] += val * val;
                    acc[2 * kHR + c] += rh * val;
                }
            }
        }
    }
    store_partials<NQ>(acc, MODE == 0 ? K.part3 : K.part6, nb);
}

// Convergence test on ||r_i||, alpha, s = r - alpha v and s^ = D^-1 s.
// Stagnation (no 0.1% decrease of a component's best ||r||^2 for win
// iterations) is handled like a breakdown, as in k_pc_s.
__global__ void __launch_bounds__(kThreads) k_h_s(HKry K, const double *__restrict__ dinv,
                                                   int64_t n, int i, int i0, double tol2, int win) {
    if (h_done(K.flag)) return;
    const int nb = gridDim.x;
    double q1[kHR], q3[kHR];
    load_partials<kHR>(K.part1, nb, q1);
    load_partials<kHR>(K.part3, nb, q3);
    double al[kHR];
    bool act[kHR];
#pragma unroll
    for (int c = 0; c < kHR; ++c) {
        act[c] = K.flag[c] == 0;
        const double rr = q1[c], rv = q3[c];
        const double rho = K.rec[((int64_t)i * kHR + c) * 4];
        al[c] = rho / rv;
        if (!act[c]) continue;
        const double bb = K.bb[c], rhrh = K.rhrh[c];
        const bool bad = !isfinite(rr) || !isfinite(rho);
        const bool conv = !bad && (rr <= tol2 * fmax(bb, 1e-300) || rr == 0.0);
        const double *bprev = K.best + ((((i + 1) & 1) * kHR) + c) * 2;
        const bool fresh = (i == i0);
        const double best = fresh ? rr : bprev[0];
        const int best_it = fresh ? i : (int)bprev[1];
        const bool better = fresh || rr < 0.999 * best;
        const bool stall = !better && (i - best_it >= win);
        const bool brk = !bad && !conv &&
                         (!(fabs(rho) > kBreakdown * sqrt(rr * rhrh)) || !isfinite(al[c]) || stall);
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            double *rc = K.rec + ((int64_t)i * kHR + c) * 4;
            rc[1] = al[c];
            rc[3] = rr;
            double *bnext = K.best + (((i & 1) * kHR) + c) * 2;
            bnext[0] = better ? rr : best;
            bnext[1] = better ? (double)i : (double)best_it;
            if (bad) K.flag[c] = -1;
            else if (conv || brk) {
                K.flag[c] = conv ? 1 : 2;
                K.iters[c] = i;
            }
        }
        if (bad || conv || brk) act[c] = false;
    }
    if (!act[0] && !act[1]) return;
    for (int64_t it = 0;; ++it) {
        const int64_t row = row_of(it);
        if (row - threadIdx.x >= n) break;
        if (row < n) {
            const double di = dinv[row];
#pragma unroll
            for (int c = 0; c < kHR; ++c) {
                if (!act[c]) continue;
                const int64_t o = c * n + row;
                const double sv = K.r[o] - al[c] * K.v[o];
                K.s[o] = sv;
                K.sh[o] = di * sv;
            }
        }
    }
}

// ------------------------------------------------ viscous Jacobi sweeps --
// When the Jacobi iteration matrix of H has a small infinity norm (max over
// rows of |1/h_ii| sum_{j != i} |h_ij|, at most kJacobiMax; H = I - a D_Lap
// with a small a), the viscous solve runs plain Jacobi sweeps: one product
// per sweep and no inner products to wait for, each sweep contracting the
// error by that norm or better.  Sweep i: x_{i+1} = x_i + D^-1 (b - H x_i)
// for both components, with block partials of ||b - H x_i||^2 and ||b||^2;
// sweep i + 1 first reduces them and stops the iteration (flag) once x_i
// passes the test, so the residual tested is the true one.
constexpr double kJacobiMax = 0.25;
struct JKry {
    double *x[2];   // [N][2] iterates by parity, components interleaved so that
                    // a gathered neighbour is one 16-byte load
    const double *x0;  // [2][N] the caller's initial guess (iterate 0)
    double *part;   // [2 parities][2 kHR][kMaxBlocks]
    double *bb;     // ||b||^2 per component
    int *flag;      // flag, then the index of the accepted iterate
};

struct GatherI2 {
    static constexpr int NV = 2;
    const double2 *x;
    __device__ __forceinline__ void operator()(int j, double (&v)[2]) const {
        const double2 t = x[j];
        v[0] = t.x;
        v[1] = t.y;
    }
};

template <int KT, bool FIRST>
__global__ void __launch_bounds__(kThreads) k_h_jac(EllM A, const double *__restrict__ b, JKry J,
                                                     int i, double tol2) {
    const int nb = gridDim.x;
    const int fl = J.flag[0];
    double q[2 * kHR] = {};
    if (i > 0) {
        const double *pp = J.part + (int64_t)((i - 1) & 1) * 2 * kHR * kMaxBlocks;
        for (int bk = threadIdx.x; bk < nb; bk += blockDim.x)
#pragma unroll
            for (int c = 0; c < 2 * kHR; ++c) q[c] += pp[(int64_t)c * kMaxBlocks + bk];
    }
    if (fl != 0) return;
    if (i > 0) {
        __shared__ double lds[2 * kHR * (kThreads / 64)];
        rbf::block_sum<2 * kHR>(q, lds);
        bool conv = true, bad = false;
#pragma unroll
        for (int c = 0; c < kHR; ++c) {
            bad = bad || !isfinite(q[c]);
            conv = conv && (q[c] <= tol2 * fmax(q[kHR + c], 1e-300) || q[c] == 0.0);
        }
        if (bad || conv) {
            if (blockIdx.x == 0 && threadIdx.x == 0) {
#pragma unroll
                for (int c = 0; c < kHR; ++c) J.bb[c] = q[kHR + c];
                J.flag[1] = i - 1;
                J.flag[0] = bad ? -1 : 1;
            }
            return;
        }
    }
    // Iterate i: the caller's [2][N] guess for i = 0, else J.x[i & 1].
    const double2 *xin = reinterpret_cast<const double2 *>(J.x[i & 1]);
    double2 *xout = reinterpret_cast<double2 *>(J.x[(i & 1) ^ 1]);
    double acc[2 * kHR] = {};
    for (int64_t it = 0;; ++it) {
        const int64_t row = row_of(it);
        if (row - threadIdx.x >= A.n) break;
        if (row < A.n) {
            double ax[1][kHR] = {};
            const double *ws[1] = {A.w};
            double xs[kHR];
            if constexpr (FIRST) {
                rbf::ell_row<KT, 1>(A.idx, ws, A.n, row, A.k, GatherN<kHR>{J.x0, A.n}, ax);
                xs[0] = J.x0[row];
                xs[1] = J.x0[A.n + row];
            } else {
                rbf::ell_row<KT, 1>(A.idx, ws, A.n, row, A.k, GatherI2{xin}, ax);
                const double2 t = xin[row];
                xs[0] = t.x;
                xs[1] = t.y;
            }
            const double di = A.dinv[row];
            double xn[kHR];
#pragma unroll
            for (int c = 0; c < kHR; ++c) {
                const double bv = b[c * A.n + row], rv = bv - ax[0][c];
                xn[c] = xs[c] + di * rv;
                acc[c] += rv * rv;
                acc[kHR + c] += bv * bv;
            }
            xout[row] = make_double2(xn[0], xn[1]);
        }
    }
    __shared__ double lds2[2 * kHR * (kThreads / 64)];
    rbf::block_sum<2 * kHR>(acc, lds2);
    if (threadIdx.x == 0) {
        double *pp = J.part + (int64_t)(i & 1) * 2 * kHR * kMaxBlocks;
#pragma unroll
        for (int c = 0; c < 2 * kHR; ++c) pp[(int64_t)c * kMaxBlocks + blockIdx.x] = acc[c];
    }
}

// The same sweep for 28-entry stencils with two lanes per row: blocks of
// 2 kThreads threads on the same grid and rows per block, so the block
// partial sums keep their count; lanes l and l + 32 of a wave take the two
// halves of row l's stencil.
template <bool FIRST>
__global__ void __launch_bounds__(2 * kThreads) k_h_jac2(EllM A, const double *__restrict__ b,
                                                        JKry J, int i, double tol2) {
    constexpr int NW = 2 * kThreads / 64;
    __shared__ double lds[2 * kHR * NW];
    const int nb = gridDim.x;
    const int fl = J.flag[0];
    double q[2 * kHR] = {};
    if (i > 0) {
        const double *pp = J.part + (int64_t)((i - 1) & 1) * 2 * kHR * kMaxBlocks;
        for (int bk = threadIdx.x; bk < nb; bk += blockDim.x)
#pragma unroll
            for (int c = 0; c < 2 * kHR; ++c) q[c] += pp[(int64_t)c * kMaxBlocks + bk];
    }
    if (fl != 0) return;
    if (i > 0) {
        rbf::block_sum<2 * kHR>(q, lds);
        bool conv = true, bad = false;
#pragma unroll
        for (int c = 0; c < kHR; ++c) {
            bad = bad || !isfinite(q[c]);
            conv = conv && (q[c] <= tol2 * fmax(q[kHR + c], 1e-300) || q[c] == 0.0);
        }
        if (bad || conv) {
            if (blockIdx.x == 0 && threadIdx.x == 0) {
#pragma unroll
                for (int c = 0; c < kHR; ++c) J.bb[c] = q[kHR + c];
                J.flag[1] = i - 1;
                J.flag[0] = bad ? -1 : 1;
            }
            return;
        }
    }
    const double2 *xin = reinterpret_cast<const double2 *>(J.x[i & 1]);
    double2 *xout = reinterpret_cast<double2 *>(J.x[(i & 1) ^ 1]);
    const int lane = threadIdx.x & 63, half = lane >> 5, wv = threadIdx.x >> 6;
    const int64_t bx = rbf::xcd_block(blockIdx.x, nb);
    double acc[2 * kHR] = {};
#pragma unroll 1
    for (int64_t it = 0;; ++it) {
        if ((bx + it * nb) * kThreads >= A.n) break;
        const int64_t row = (bx + it * nb) * kThreads + wv * 32 + (lane & 31);
        const int64_t rr = (row < A.n) ? row : A.n - 1;
        double ax[kHR] = {};
        if constexpr (FIRST)
            rbf::ell_half_row<28>(A.idx, A.w, A.n, rr, half, GatherN<kHR>{J.x0, A.n}, ax);
        else
            rbf::ell_half_row<28>(A.idx, A.w, A.n, rr, half, GatherI2{xin}, ax);
#pragma unroll
        for (int c = 0; c < kHR; ++c) ax[c] += __shfl_xor(ax[c], 32, 64);
        if (half == 0 && row < A.n) {
            double xs[kHR];
            if constexpr (FIRST) {
                xs[0] = J.x0[row];
                xs[1] = J.x0[A.n + row];
            } else {
                const double2 t = xin[row];
                xs[0] = t.x;
                xs[1] = t.y;
            }
            const double di = A.dinv[row];
            double xn[kHR];
#pragma unroll
            for (int c = 0; c < kHR; ++c) {
                const double bv = b[c * A.n + row], rv = bv - ax[c];
                xn[c] = xs[c] + di * rv;
                acc[c] += rv * rv;
                acc[kHR + c] += bv * bv;
            }
            xout[row] = make_double2(xn[0], xn[1]);
        }
    }
    rbf::block_sum<2 * kHR>(acc, lds);
    if (threadIdx.x == 0) {
        double *pp = J.part + (int64_t)(i & 1) * 2 * kHR * kMaxBlocks;
#pragma unroll
        for (int c = 0; c < 2 * kHR; ++c) pp[(int64_t)c * kMaxBlocks + blockIdx.x] = acc[c];
    }
}

// x ([2][N]) from an interleaved iterate ([N][2]).
__global__ void k_h_deint(int64_t n, const double2 *__restrict__ xi, double *__restrict__ x) {
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= n) return;
    const double2 t = xi[r];
    x[r] = t.x;
    x[n + r] = t.y;
}

// Block maxima of |1/h_ii| sum_{j != i} |h_ij| (the Jacobi bound above).
__global__ void __launch_bounds__(256) k_jacobi_bound(int64_t n, int k, const int *__restrict__ idx,
                                                      const double *__restrict__ hw,
                                                      const double *__restrict__ dinv,
                                                      double *__restrict__ part) {
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    double q = 0.0;
    if (r < n) {
        double off = 0.0;
        for (int s = 0; s < k; ++s) {
            const int64_t o = (int64_t)s * n + r;
            if (idx[o] != r) off += fabs(hw[o]);
        }
        q = fabs(dinv[r]) * off;
    }
    __shared__ double m[256];
    m[threadIdx.x] = q;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) m[threadIdx.x] = fmax(m[threadIdx.x], m[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = m[0];
}

// ---------------------------------------------------------- step kernels --
// Stage 1: C(q) = -(u o D_x q + v o D_y q), u* = u + dt (3/2 C_j - 1/2 C_{j-1}).
template <int KT>
__global__ void __launch_bounds__(kThreads) k_advect(int64_t n, int k, const int *__restrict__ idx,
                                                      const double *__restrict__ wdx,
                                                      const double *__restrict__ wdy,
                                                      const double *__restrict__ u,
                                                      const double *__restrict__ v,
                                                      const double *__restrict__ cu_prev,
                                                      const double *__restrict__ cv_prev,
                                                      int first, double dt, double *__restrict__ us,
                                                      double *__restrict__ vs,
                                                      double *__restrict__ cu,
                                                      double *__restrict__ cv) {
    const int64_t r = (int64_t)rbf::xcd_block(blockIdx.x, gridDim.x) * kThreads + threadIdx.x;
    if (r >= n) return;
    double acc[2][2] = {};
    const double *ws[2] = {wdx, wdy};
    rbf::ell_row<KT, 2>(idx, ws, n, r, k, Gather2{u, v}, acc);
    const double ui = u[r], vi = v[r];
    const double cun = -(ui * acc[0][0] + vi * acc[1][0]);
    const double cvn = -(ui * acc[0][1] + vi * acc[1][1]);
    const double cup = first ? cun : cu_prev[r];
    const double cvp = first ? cvn : cv_prev[r];
    us[r] = ui + dt * (1.5 * cun - 0.5 * cup);
    vs[r] = vi + dt * (1.5 * cvn - 0.5 * cvp);
    cu[r] = cun;
    cv[r] = cvn;
}

// Stage 2 right-hand side on interior rows: (I + a D_Lap) u*, and the same
// for v; the initial guess of the solve is the right-hand side.
template <int KT>
__global__ void __launch_bounds__(kThreads) k_helm_rhs(int64_t n, int k, const int *__restrict__ idx,
                                                        const double *__restrict__ wlap, double a,
                                                        const double *__restrict__ us,
                                                        const double *__restrict__ vs,
                                                        double *__restrict__ rhs,
                                                        double *__restrict__ x0) {
    const int64_t r = (int64_t)rbf::xcd_block(blockIdx.x, gridDim.x) * kThreads + threadIdx.x;
    if (r >= n) return;
    double acc[1][2] = {};
    const double *ws[1] = {wlap};
    rbf::ell_row<KT, 1>(idx, ws, n, r, k, Gather2{us, vs}, acc);
    const double ru = us[r] + a * acc[0][0];
    const double rv = vs[r] + a * acc[0][1];
    rhs[r] = ru;
    rhs[n + r] = rv;
    x0[r] = ru;
    x0[n + r] = rv;
}

// Open boundary rows (channel flows; the cavity has none).  Tag
// RBF_VTAG_OUTFLOW: convective outflow dq/dt + uc dq/dx = 0, explicit Euler
// from step j: q_bc = q_j - dt uc (D_x^VV q_j) for q = u, v.  Tag
// RBF_VTAG_SYMMETRY: v_bc = 0 and u_bc solves the node's own D_y^VV row for
// du/dy = 0 with the neighbours' values at step j.
struct OpenBc {
    const int8_t *vtag;     // [N] V-node tags (nullptr: no open rows)
    const int *idx;         // (V,V) stencils
    const double *wdx, *wdy;
    const double *u, *v;    // state at step j
    double uc;              // convection velocity of the outflow rows
};

template <int KT>
__device__ __forceinline__ void open_bc_values(const OpenBc &B, int64_t n, int k, int64_t r,
                                               double &ub, double &vb, double dt) {
    const int t = B.vtag[r];
    if (t == RBF_VTAG_OUTFLOW) {
        double acc[1][2] = {};
        const double *ws[1] = {B.wdx};
        rbf::ell_row<KT, 1>(B.idx, ws, n, r, k, Gather2{B.u, B.v}, acc);
        ub = B.u[r] - dt * B.uc * acc[0][0];
        vb = B.v[r] - dt * B.uc * acc[0][1];
    } else if (t == RBF_VTAG_SYMMETRY) {
        double diag = 0.0, off = 0.0;
        for (int q = 0; q < k; ++q) {
            const int j = B.idx[(int64_t)q * n + r];
            const double w = B.wdy[(int64_t)q * n + r];
            if (j == r) diag += w;
            else off = fma(w, B.u[j], off);
        }
        ub = -off / diag;
        vb = 0.0;
    }
}

// Kim-Moin wall values (eq. (21)): u** = u_bc + dt D_x^VP p~_j, v** likewise,
// with u_bc, v_bc of the open rows computed from the state at step j.
template <int KT>
__global__ void __launch_bounds__(kThreads) k_wall_rhs(int64_t nwall, const int *__restrict__ rows,
                                                        int64_t n, int k, const int *__restrict__ idx,
                                                        const double *__restrict__ wdx,
                                                        const double *__restrict__ wdy,
                                                        const double *__restrict__ pt,
                                                        const double *__restrict__ u_bc,
                                                        const double *__restrict__ v_bc, double dt,
                                                        double *__restrict__ rhs,
                                                        double *__restrict__ x0, OpenBc B) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= nwall) return;
    const int64_t r = rows[i];
    double acc[2][1] = {};
    const double *ws[2] = {wdx, wdy};
    rbf::ell_row<KT, 2>(idx, ws, n, r, k, GatherN<1>{pt, 0}, acc);
    double ub = u_bc[r], vb = v_bc[r];
    if (B.vtag) open_bc_values<KT>(B, n, k, r, ub, vb, dt);
    const double ru = ub + dt * acc[0][0], rv = vb + dt * acc[1][0];
    rhs[r] = ru;
    rhs[n + r] = rv;
    x0[r] = ru;
    x0[n + r] = rv;
}

// Stage 3a: F = D_x^PV u** + D_y^PV v**; Poisson right-hand side F/dt on
// interior rows (times the row scaling of the stored Poisson matrix), 0 on
// wall rows.
template <int KT>
__global__ void __launch_bounds__(kThreads) k_divergence(int64_t m, int k, const int *__restrict__ idx,
                                                          const double *__restrict__ wdx,
                                                          const double *__restrict__ wdy,
                                                          const double *__restrict__ uss,
                                                          const double *__restrict__ vss,
                                                          const int8_t *__restrict__ ptag,
                                                          double inv_dt,
                                                          const double *__restrict__ rowscale,
                                                          double *__restrict__ rhs) {
    const int64_t r = (int64_t)rbf::xcd_block(blockIdx.x, gridDim.x) * kThreads + threadIdx.x;
    if (r >= m) return;
    double acc[2][2] = {};
    const double *ws[2] = {wdx, wdy};
    rbf::ell_row<KT, 2>(idx, ws, m, r, k, Gather2{uss, vss}, acc);
    const double F = acc[0][0] + acc[1][1];
    rhs[r] = (ptag[r] == 0) ? rowscale[r] * (F * inv_dt) : 0.0;
}

// Stage 3c (pressure): p = p~ - a D_Lap^PP p~.
template <int KT>
__global__ void __launch_bounds__(kThreads) k_pressure(int64_t m, int k, const int *__restrict__ idx,
                                                        const double *__restrict__ wlap, double a,
                                                        const double *__restrict__ pt,
                                                        double *__restrict__ p) {
    const int64_t r = (int64_t)rbf::xcd_block(blockIdx.x, gridDim.x) * kThreads + threadIdx.x;
    if (r >= m) return;
    double acc[1][1] = {};
    const double *ws[1] = {wlap};
    rbf::ell_row<KT, 1>(idx, ws, m, r, k, GatherN<1>{pt, 0}, acc);
    p[r] = pt[r] - a * acc[0][0];
}

// Stage 3c (velocity): u = u** - dt D_x^VP p~, v = v** - dt D_y^VP p~, all rows.
template <int KT>
__global__ void __launch_bounds__(kThreads) k_correct(int64_t n, int k, const int *__restrict__ idx,
                                                       const double *__restrict__ wdx,
                                                       const double *__restrict__ wdy, double dt,
                                                       const double *__restrict__ pt,
                                                       const double *__restrict__ uvss,
                                                       double *__restrict__ u, double *__restrict__ v) {
    const int64_t r = (int64_t)rbf::xcd_block(blockIdx.x, gridDim.x) * kThreads + threadIdx.x;
    if (r >= n) return;
    double acc[2][1] = {};
    const double *ws[2] = {wdx, wdy};
    rbf::ell_row<KT, 2>(idx, ws, n, r, k, GatherN<1>{pt, 0}, acc);
    u[r] = uvss[r] - dt * acc[0][0];
    v[r] = uvss[n + r] - dt * acc[1][0];
}

// ----------------------------------------------- system matrix assembly --
// H = I - a D_Lap on interior V rows, identity on wall rows.
__global__ void k_build_helmholtz(int64_t n, int k, const int *__restrict__ idx,
                                  const double *__restrict__ lap, const int8_t *__restrict__ tag,
                                  double a, double *__restrict__ hw, double *__restrict__ dinv,
                                  int *__restrict__ err) {
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= n) return;
    const bool wall = tag[r] != 0;
    double diag = 0.0;
    bool self = false;
    for (int s = 0; s < k; ++s) {
        const int64_t o = (int64_t)s * n + r;
        const bool me = idx[o] == r;
        double wv = wall ? 0.0 : -a * lap[o];
        if (me) {
            wv += 1.0;
            diag = wv;
            self = true;
        }
        hw[o] = wv;
    }
    if (!self) atomicOr(err, 1);
    dinv[r] = (diag != 0.0) ? 1.0 / diag : 1.0;
}

// Poisson rows: D_Lap^PP (interior), n_x D_x^PP + n_y D_y^PP (wall), stored
// row-scaled: interior rows by -1/||row||_2, wall rows by +1/||row||_2, so
// the scaled operator is -Lap with outward-normal Neumann rows, whose
// spectrum lies in the right half-plane.  RBF-FD self-weights do not have a
// fixed sign on scattered nodes, so Jacobi scaling would make the spectrum
// indefinite; BiCGSTAB on the row-scaled matrix runs unpreconditioned
// (dinv = 1).  rowscale[r] scales the right-hand side; u1 = rowscale on
// interior rows (0 on wall rows) is the uniform-source column of the border.
__global__ void k_build_poisson(int64_t m, int k, const int *__restrict__ idx,
                                const double *__restrict__ lap, const double *__restrict__ dx,
                                const double *__restrict__ dy, const int8_t *__restrict__ tag,
                                const double *__restrict__ nrm, double *__restrict__ pw,
                                double *__restrict__ dinv, double *__restrict__ rowscale,
                                double *__restrict__ u1, int *__restrict__ err) {
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= m) return;
    const bool wall = tag[r] != 0;
    const double nx = nrm[r], ny = nrm[m + r];
    bool self = false;
    double ss = 0.0;
    for (int s = 0; s < k; ++s) {
        const int64_t o = (int64_t)s * m + r;
        if (idx[o] == r) self = true;
        const double wv = wall ? nx * dx[o] + ny * dy[o] : lap[o];
        ss += wv * wv;
        pw[o] = wv;
    }
    if (!self || !(ss > 0.0)) atomicOr(err, 2);
    const double sc = (wall ? 1.0 : -1.0) / sqrt(ss);
    for (int s = 0; s < k; ++s) pw[(int64_t)s * m + r] *= sc;
    rowscale[r] = sc;
    u1[r] = wall ? 0.0 : sc;
    dinv[r] = 1.0;
}

// Warm start of the pressure solve by extrapolation in time from the
// previous solutions: ORDER 1: x0 = 2 x_j - x_{j-1}; ORDER 2:
// x0 = 3 x_j - 3 x_{j-1} + x_{j-2}; ORDER 3: x0 = 4 x_j - 6 x_{j-1} +
// 4 x_{j-2} - x_{j-3}; the history shifts by one step.
template <int ORDER>
__global__ void k_extrapolate(int64_t n, double *__restrict__ x, double *__restrict__ x1,
                              double *__restrict__ x2, double *__restrict__ x3) {
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= n) return;
    const double t = x[r], t1 = x1[r];
    if constexpr (ORDER == 3) {
        const double t2 = x2[r];
        x[r] = 4.0 * t - 6.0 * t1 + 4.0 * t2 - x3[r];
        x3[r] = t2;
    } else if constexpr (ORDER == 2) {
        const double t2 = x2[r];
        x[r] = 3.0 * t - 3.0 * t1 + t2;
        x3[r] = t2;
    } else {
        x[r] = 2.0 * t - t1;
    }
    x2[r] = t1;
    x1[r] = t;
}

// Initial guess of the viscous solve from the previous solutions h0
// (latest), h1, h2, h3 (ORDER 1-4: constant, linear, quadratic, cubic in
// time).
template <int ORDER>
__global__ void k_guess(int64_t n, double *__restrict__ x, const double *__restrict__ h0,
                        const double *__restrict__ h1, const double *__restrict__ h2,
                        const double *__restrict__ h3) {
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= n) return;
    if constexpr (ORDER == 1) x[r] = h0[r];
    else if constexpr (ORDER == 2) x[r] = 2.0 * h0[r] - h1[r];
    else if constexpr (ORDER == 3) x[r] = 3.0 * h0[r] - 3.0 * h1[r] + h2[r];
    else x[r] = 4.0 * h0[r] - 6.0 * h1[r] + 4.0 * h2[r] - h3[r];
}

// rhs_scaled = rowscale o rhs (for rbf_solve_pressure).
__global__ void k_scale(int64_t n, const double *__restrict__ sc, const double *__restrict__ a,
                        double *__restrict__ b) {
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r < n) b[r] = sc[r] * a[r];
}

__global__ void k_wall_list(int64_t n, const int8_t *__restrict__ tag, int *__restrict__ list,
                            int *__restrict__ count) {
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= n || tag[r] == 0) return;
    list[atomicAdd(count, 1)] = (int)r;
}

#include "pressure_aux.h"
#include "adjoint.h"
#include "viscous_mixed.h"

}  // namespace

// ====================================================================== host
struct rbf_solver {
    hipStream_t st = nullptr;
    int device = 0;  // current device at creation (the stream's device)
    int64_t N = 0, M = 0;
    int k = 0;
    double re = 0, dt = 0, a = 0, rtol_h = 0, rtol_p = 0;
    int maxit_h = 0, maxit_p = 0;
    int64_t nwall = 0;
    // operators
    int *idx_vv = nullptr, *idx_pv = nullptr, *idx_pp = nullptr, *idx_vp = nullptr;
    double *vv_dx = nullptr, *vv_dy = nullptr, *vv_lap = nullptr, *pv_dx = nullptr,
           *pv_dy = nullptr, *pp_lap = nullptr, *vp_dx = nullptr, *vp_dy = nullptr;
    double *h_w = nullptr, *h_dinv = nullptr, *p_w = nullptr, *p_dinv = nullptr,
           *p_rowscale = nullptr, *p_rhs_tmp = nullptr, *p_u1 = nullptr, *p_warm = nullptr,
           *p_prev = nullptr, *p_prev2 = nullptr, *p_prev3 = nullptr;
    int have_prev = 0;  // previous solutions held in p_prev, p_prev2 (within one rbf_step call)
    double *hh[4] = {nullptr, nullptr, nullptr, nullptr};  // previous viscous solutions [2][N], latest first
    int have_h = 0;
    double p_vscale = 0.0;
    int8_t *p_tag = nullptr;
    int *wall_rows = nullptr;
    int8_t *v_tag_open = nullptr;  // [N] V tags when open boundary rows exist
    struct Forces {  // body rows and quadrature of rbf_solver_forces (cached)
        bool ready = false;
        int tag = 0, np = 0, nv = 0, cap = 0;
        double cx = 0, cy = 0, radius = 0;
        int *prow = nullptr, *vrow = nullptr;
        double *pq = nullptr, *vq = nullptr, *out = nullptr;
    } forces;
    double u_conv = 0.0;           // convection velocity of outflow rows
    double *u_bc = nullptr, *v_bc = nullptr;
    double *v_hmin = nullptr;    // [N] nearest stencil-neighbour distance (CFL)
    double *diag_part = nullptr; // [5][kMaxBlocks] diagnostics partials
    int64_t n_interior_p = 0;
    // state (committed) and step workspace
    double *u = nullptr, *v = nullptr, *pt = nullptr, *p = nullptr, *cu = nullptr, *cv = nullptr;
    double *un = nullptr, *vn = nullptr, *ptn = nullptr, *pn = nullptr, *cun = nullptr,
           *cvn = nullptr;
    double *us = nullptr, *vs = nullptr, *hrhs = nullptr, *uvss = nullptr, *prhs = nullptr;
    // Krylov workspaces: Helmholtz (2 RHS over N), Poisson (1 RHS over M)
    KDev kp{};
    double *rpart = nullptr;
    int last_iters_h = 0, last_iters_p = 0;
    int p_hist[3] = {0, 0, 0};  // iteration counts of the last pressure solves (ring)
    int p_nhist = 0, p_pos = 0;
    // optional sampling of the Poisson SpMV duration with HIP events
    // Sampled kernel durations (rbf_solver_profile): event pairs recorded
    // around sampled launches, read after the solver's next stream sync.
    static constexpr int kProfPairs = 64;
    int prof_every = 0;
    int64_t prof_launches = 0, prof_count[RBF_PROF_N] = {};
    double prof_ms[RBF_PROF_N] = {};
    std::vector<hipEvent_t> prof_ev[RBF_PROF_N];
    int prof_pending[RBF_PROF_N] = {};
    // Arnoldi step of each pending pair (-1: not an FGMRES step), so that
    // launches made after convergence (they exit at the flag test) are not
    // counted; prof_tag_now is the tag given to the pairs being recorded.
    int prof_tag[RBF_PROF_N][kProfPairs] = {};
    int prof_tag_now = -1;
    // lattice preconditioner of the pressure system
    bool pc_on = false;
    bool mixed = false;  // RBF_PRECISION_MIXED
    HKry hk{};           // viscous solve with explicit vectors
    JKry jk{};           // viscous solve by Jacobi sweeps
    bool h_jacobi = false;  // Jacobi bound of H <= kJacobiMax
    HMix hm{};           // mixed precision: FP32 sweeps inside FP64 refinement
    bool h_mixed = false;
    double h_bound = 0.0;
    Lat lat{};
    PKry pk{};
    // two-level auxiliary-lattice preconditioner with FGMRES (general nodes)
    bool aux_on = false;
    int aux_K = 0;             // cells per side of the auxiliary lattice
    AuxOps<double> ax64{};
    AuxOps<float> ax32{};
    FgDev<double> fg64{};
    FgDev<float> fg32{};
    float *p_w32 = nullptr;    // FP32 Poisson weights (mixed precision)
    // adjoint step (rbf_adjoint_step): transposed operators and work vectors,
    // built at its first call
    struct Adj {
        bool ready = false;
        int64_t *cp_vv = nullptr, *cp_vp = nullptr, *cp_pv = nullptr, *cp_pp = nullptr;
        int *src_vv = nullptr, *src_vp = nullptr, *src_pv = nullptr, *src_pp = nullptr;
        double *dxT_vv = nullptr, *dyT_vv = nullptr, *lapT_vv = nullptr, *dxT_vp = nullptr,
               *dyT_vp = nullptr, *dxT_pv = nullptr, *dyT_pv = nullptr, *aT_pp = nullptr;
        int8_t *vtag = nullptr;  // 1 on wall V rows
        double *vn[20] = {};     // work vectors over V rows
        double *pm[8] = {};      // work vectors over P rows
        double *kr[7] = {};      // Krylov vectors (max(N, M))
        double *part = nullptr;
    } adj;
    // pinned host buffers
    int *hflag = nullptr;
    double *hred = nullptr;
    std::vector<void *> allocs;
};

namespace {

// Event pair for a sampled launch in profiling slot q (false when the
// slot's pairs are all pending).  The launch is made with
// hipExtLaunchKernelGGL, which stamps the kernel's own start and end.
bool prof_pair(rbf_solver *S, int q, hipEvent_t &e0, hipEvent_t &e1) {
    if (S->prof_pending[q] >= rbf_solver::kProfPairs || S->prof_ev[q].empty()) return false;
    e0 = S->prof_ev[q][2 * S->prof_pending[q]];
    e1 = S->prof_ev[q][2 * S->prof_pending[q] + 1];
    S->prof_tag[q][S->prof_pending[q]] = S->prof_tag_now;
    ++S->prof_pending[q];
    return true;
}
// After a stream synchronisation: accumulate the recorded pairs; pairs of
// FGMRES steps at or after steps_done (launched after convergence, so they
// exited at the flag test) are dropped.
void prof_flush(rbf_solver *S, int steps_done = 1 << 30) {
    for (int q = 0; q < RBF_PROF_N; ++q) {
        const int per = 1;
        for (int e = 0; e < S->prof_pending[q]; ++e) {
            float ms = 0.f;
            if (S->prof_tag[q][e] >= steps_done) continue;
            if (hipEventElapsedTime(&ms, S->prof_ev[q][2 * e], S->prof_ev[q][2 * e + 1]) ==
                hipSuccess) {
                S->prof_ms[q] += ms;
                S->prof_count[q] += per;
            }
        }
        S->prof_pending[q] = 0;
    }
}

rbf_status dalloc(rbf_solver *S, void **p, size_t bytes) {
    hipError_t e = hipMalloc(p, bytes ? bytes : 8);
    if (e != hipSuccess) {
        rbf::set_error("rbf_solver: hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
        return RBF_E_NOMEM;
    }
    S->allocs.push_back(*p);
    return RBF_OK;
}

#define ALLOC(ptr, count)                                                          \
    do {                                                                           \
        rbf_status rc_ = dalloc(S, (void **)&(ptr), sizeof(*(ptr)) * (size_t)(count)); \
        if (rc_ != RBF_OK) return rc_;                                             \
    } while (0)

int nblocks_rows(int64_t n) {
    return (int)std::min<int64_t>(kMaxBlocks, (n + kThreads - 1) / kThreads);
}

rbf_status alloc_krylov(rbf_solver *S, KDev &K, int nr, int64_t n, int maxit) {
    const int64_t len = (int64_t)nr * n;
    for (int q = 0; q < 2; ++q) {
        ALLOC(K.q[q], 4 * len);
        ALLOC(K.partA[q], 5 * nr * kMaxBlocks);
    }
    ALLOC(K.rh, len);
    ALLOC(K.partB, 4 * nr * kMaxBlocks);
    ALLOC(K.partX, nr * kMaxBlocks);
    ALLOC(K.rec, (int64_t)(maxit + 2) * nr * 4);
    ALLOC(K.bb, nr);
    ALLOC(K.rhrh, nr);
    ALLOC(K.flag, nr);
    ALLOC(K.iters, nr);
    return RBF_OK;
}

// BiCGSTAB on A x = b for NR stacked right-hand sides (x: initial guess in,
// solution out).  JAC: Jacobi preconditioning with A.dinv.
template <int NR, bool JAC>
rbf_status bicgstab(rbf_solver *S, KDev &K, EllM A, const double *b, double *x, double tol,
                    int maxit, int &last_iters, rbf_solve_stats *stats) {
    hipStream_t st = S->st;
    const int nb = nblocks_rows(A.n);
    const double tol2 = tol * tol;
    const bool k28 = A.k == 28;
    const dim3 grid(nb), block(kThreads);
#define KRY(kern, ...)                                                                         \
    do {                                                                                       \
        if (k28) hipLaunchKernelGGL((kern<NR, 28, JAC>), grid, block, 0, st, __VA_ARGS__);     \
        else hipLaunchKernelGGL((kern<NR, 0, JAC>), grid, block, 0, st, __VA_ARGS__);          \
    } while (0)
#define KRY2(kern, ...)                                                                        \
    do {                                                                                       \
        if (k28) hipLaunchKernelGGL((kern<NR, 28>), grid, block, 0, st, __VA_ARGS__);          \
        else hipLaunchKernelGGL((kern<NR, 0>), grid, block, 0, st, __VA_ARGS__);               \
    } while (0)
    auto init = [&](int i) {
        if (A.u1) hipLaunchKernelGGL((k_sum<NR>), grid, block, 0, st, A.n, x, K.partX);
        KRY2(k_kry_init, A, b, x, K, i & 1);
    };
    init(0);
    int it = 0, i0 = 0, restarts = 0;
    rbf_status rc = RBF_OK;
    int batch = std::max(4, last_iters > 0 ? last_iters - 1 : 8);
    bool done = false;
    while (!done) {
        const int stop = std::min(maxit + 1, it + batch);
        for (; it < stop; ++it) {
            const int par = it & 1;
            const bool sample =
                NR == 1 && S->prof_every > 0 && (S->prof_launches++ % S->prof_every) == 0;
            hipEvent_t e0 = nullptr, e1 = nullptr;
            if (sample && prof_pair(S, RBF_PROF_SPMV, e0, e1)) {
                if (k28) hipExtLaunchKernelGGL((k_kry_a<NR, 28, JAC>), grid, block, 0, st, e0, e1, 0,
                                               A, K, x, it, i0, par);
                else hipExtLaunchKernelGGL((k_kry_a<NR, 0, JAC>), grid, block, 0, st, e0, e1, 0,
                                           A, K, x, it, i0, par);
            } else {
                KRY(k_kry_a, A, K, x, it, i0, par);
            }
            KRY(k_kry_b, A, K, it, par, tol2);
        }
        RBF_CHECK_LAUNCH();
        RBF_HIP(hipMemcpyAsync(S->hflag, K.flag, NR * sizeof(int), hipMemcpyDeviceToHost, st));
        RBF_HIP(hipMemcpyAsync(S->hflag + kMaxNR, K.iters, NR * sizeof(int), hipMemcpyDeviceToHost, st));
        RBF_HIP(hipStreamSynchronize(st));
        prof_flush(S);
        done = true;
        bool restart = false;
        int brk_at = it;
        for (int c = 0; c < NR; ++c) {
            if (S->hflag[c] == 0) done = false;
            if (S->hflag[c] == 2) {
                restart = true;
                brk_at = std::min(brk_at, S->hflag[kMaxNR + c]);
            }
        }
        if (restart && it <= maxit && restarts < 50) {
            // Breakdown: restart from the current iterate with rh = r.  Kernels
            // launched after the flag was set did nothing, so the iteration
            // count resumes where the breakdown occurred.
            ++restarts;
            it = i0 = brk_at;
            init(it);
            done = false;
            continue;
        }
        if (!done && it > maxit) break;
        batch = std::max(4, std::min(64, (it - i0) / 4));
    }
    // Final statistics: true residual.
    if (A.u1) hipLaunchKernelGGL((k_sum<NR>), grid, block, 0, st, A.n, x, K.partX);
    KRY2(k_resid, A, b, x, S->rpart, K.partX);
    RBF_CHECK_LAUNCH();
    RBF_HIP(hipMemcpyAsync(S->hred, S->rpart, (size_t)NR * nb * sizeof(double), hipMemcpyDeviceToHost, st));
    RBF_HIP(hipMemcpyAsync(S->hred + kMaxNR * kMaxBlocks, K.bb, NR * sizeof(double), hipMemcpyDeviceToHost, st));
    RBF_HIP(hipStreamSynchronize(st));
#undef KRY
#undef KRY2
    int maxi = 0;
    for (int c = 0; c < NR; ++c) {
        double rr = 0.0;
        for (int bidx = 0; bidx < nb; ++bidx) rr += S->hred[c * nb + bidx];
        const double bb = S->hred[kMaxNR * kMaxBlocks + c];
        const int f = S->hflag[c];
        const int iters = (f == 1) ? S->hflag[kMaxNR + c] : it;
        maxi = std::max(maxi, iters);
        if (stats) {
            stats[c].iterations = iters;
            stats[c].converged = (f == 1);
            stats[c].rel_residual = (bb > 0.0) ? std::sqrt(rr / bb) : std::sqrt(rr);
            stats[c].restarts = restarts;
            stats[c].final_flag = f;
        }
        if (f == -1) {
            rbf::set_error("BiCGSTAB: non-finite value (rhs %d, iteration %d)", c, it);
            rc = RBF_E_NAN;
        } else if ((f == 0 || f == 2) && rc == RBF_OK) {
            rbf::set_error("BiCGSTAB: no convergence (rhs %d, %d of %d iterations, %d restarts, flag %d)",
                           c, it, maxit, restarts, f);
            rc = RBF_E_NOCONV;
        }
    }
    last_iters = maxi;
    return rc;
}

// One application of the lattice preconditioner's interior solve:
// T = Q^-1 X, tridiagonal solves along y per x-mode, Z = Q W.
rbf_status pc_apply(rbf_solver *S, bool sample = false) {
    const dim3 g(S->lat.ntiles), b(64 * kGemmWaves);
    const dim3 gt(S->lat.n), bt(64);
    // A sample times the first product (its own start and end stamps).
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const bool timed = sample && prof_pair(S, RBF_PROF_GEMM, e0, e1);
    const int steps = (S->lat.n + 3) / 4;
    const bool one = (steps + kGemmWaves - 1) / kGemmWaves <= kGemmChunk;
    auto run = [&](auto tp) {
        using TP = decltype(tp);
        if (one) hipExtLaunchKernelGGL((k_pc_gemm<0, true, TP>), g, b, 0, S->st, e0, e1, 0, S->lat);
        else hipExtLaunchKernelGGL((k_pc_gemm<0, false, TP>), g, b, 0, S->st, e0, e1, 0, S->lat);
        hipLaunchKernelGGL(k_pc_tri<TP>, gt, bt, 0, S->st, S->lat);
        if (one) hipLaunchKernelGGL((k_pc_gemm<1, true, TP>), g, b, 0, S->st, S->lat);
        else hipLaunchKernelGGL((k_pc_gemm<1, false, TP>), g, b, 0, S->st, S->lat);
    };
    if (S->lat.f32) run(float{});
    else run(double{});
    (void)timed;
    return RBF_OK;
}

// Right-preconditioned BiCGSTAB on the pressure system (one right-hand side)
// with the lattice preconditioner; same contract as bicgstab<1, false>.
// Per iteration: k_pc_dir, P^-1 (k_pc_gemm, k_pc_tri, k_pc_gemm, k_pc_post),
// k_pc_av (v), k_pc_s, P^-1, k_pc_av (t).
rbf_status pbicgstab(rbf_solver *S, EllM A, const double *b, double *x, double tol, int maxit,
                     int &last_iters, rbf_solve_stats *stats) {
    hipStream_t st = S->st;
    PKry &K = S->pk;
    const Lat &L = S->lat;
    const int64_t m = A.n;
    const int nb = nblocks_rows(m);
    const dim3 grid(nb), block(kThreads);
    const double tol2 = tol * tol;
    const bool k28 = A.k == 28;
    double *partX = S->kp.partX;
    auto init = [&]() {
        if (A.u1) hipLaunchKernelGGL((k_sum<1>), grid, block, 0, st, m, x, partX);
        if (k28) hipLaunchKernelGGL((k_pc_init<28>), grid, block, 0, st, A, b, x, K, partX);
        else hipLaunchKernelGGL((k_pc_init<0>), grid, block, 0, st, A, b, x, K, partX);
    };
    auto av = [&](int mode, const double *y, double *out, hipEvent_t e0, hipEvent_t e1) {
        if (k28) {
            if (mode == 0) hipExtLaunchKernelGGL((k_pc_av<28, 0>), grid, block, 0, st, e0, e1, 0, A, K, y, out);
            else hipLaunchKernelGGL((k_pc_av<28, 1>), grid, block, 0, st, A, K, y, out);
        } else {
            if (mode == 0) hipExtLaunchKernelGGL((k_pc_av<0, 0>), grid, block, 0, st, e0, e1, 0, A, K, y, out);
            else hipLaunchKernelGGL((k_pc_av<0, 1>), grid, block, 0, st, A, K, y, out);
        }
    };
    init();
    int it = 0, i0 = 0, restarts = 0;
    rbf_status rc = RBF_OK;
    // Launch plan.  Launches after convergence exit after their first loads
    // but still cost a few microseconds each, and every batch ends with a
    // host synchronisation: the first batch stops a few iterations short of
    // the fewest among the last three solves; later batches cover the
    // iterations still needed at the residual's recent rate of decrease
    // (from the status block), or grow 2, 2, 4, 8, 16 when no rate is known
    // (after a restart, from 4).
    int expect = 0;
    for (int q = 0; q < S->p_nhist; ++q) expect = q ? std::min(expect, S->p_hist[q]) : S->p_hist[q];
    int batch = S->p_nhist ? std::max(2, expect - 4) : 8;
    int grow = 2, small = 0;
    int win = kStall;
    bool done = false;
    while (!done) {
        const int stop = std::min(maxit + 1, it + batch);
        for (; it < stop; ++it) {
            const int par = it & 1;
            const bool sample = S->prof_every > 0 && (S->prof_launches++ % S->prof_every) == 0;
            hipLaunchKernelGGL(k_pc_dir, grid, block, 0, st, K, L, x, m, it, i0);
            if ((rc = pc_apply(S, sample)) != RBF_OK) return rc;
            hipLaunchKernelGGL(k_pc_post, grid, block, 0, st, L, K, K.p[par], K.ph, m, K.partS,
                               K.part1 + nb, nb);
            hipEvent_t e0 = nullptr, e1 = nullptr;
            if (sample) prof_pair(S, RBF_PROF_SPMV, e0, e1);
            av(0, K.ph, K.v, e0, e1);
            hipLaunchKernelGGL(k_pc_s, grid, block, 0, st, K, L, m, it, i0, tol2, win);
            if ((rc = pc_apply(S)) != RBF_OK) return rc;
            hipLaunchKernelGGL(k_pc_post, grid, block, 0, st, L, K, K.s, K.sh, m, K.partS,
                               K.partGs, nb);
            av(1, K.sh, K.t, nullptr, nullptr);
        }
        RBF_CHECK_LAUNCH();
        RBF_HIP(hipMemcpyAsync(S->hflag, K.flag, 2 * sizeof(int) + 3 * sizeof(double),
                               hipMemcpyDeviceToHost, st));
        RBF_HIP(hipStreamSynchronize(st));
        prof_flush(S);
        const int f = S->hflag[0];
        const double *hs = reinterpret_cast<const double *>(S->hflag + 2);
        done = (f != 0);
        if (f == 2 && it <= maxit && restarts < 50) {
            // Breakdown: restart from the current iterate with rh = r.
            ++restarts;
            it = i0 = S->hflag[1];
            init();
            done = false;
            batch = 4;
            grow = 8;
            win = std::min(2 * win, 1 << 20);
            continue;
        }
        if (!done && it > maxit) break;
        batch = grow;
        if (++small > 1) grow = std::min(16, 2 * grow);
        // Every launched iteration ran (no flag): hs[0] is ||r||^2 at it - 1,
        // hs[1] at max(i0, it - 5).
        const int span = std::min(4, it - 1 - i0);
        if (span > 0 && hs[0] > 0.0 && hs[1] > 0.0) {
            const double rate = std::log(hs[0] / hs[1]) / span;  // per iteration
            const double need = std::log(tol2 * std::fmax(hs[2], 1e-300) / hs[0]);
            if (rate < -1e-3 && std::isfinite(rate) && std::isfinite(need))
                batch = std::max(1, std::min(8, (int)(need / rate)));
        }
    }
    if (A.u1) hipLaunchKernelGGL((k_sum<1>), grid, block, 0, st, m, x, partX);
    if (k28) hipLaunchKernelGGL((k_resid<1, 28>), grid, block, 0, st, A, b, x, S->rpart, partX);
    else hipLaunchKernelGGL((k_resid<1, 0>), grid, block, 0, st, A, b, x, S->rpart, partX);
    RBF_CHECK_LAUNCH();
    RBF_HIP(hipMemcpyAsync(S->hred, S->rpart, (size_t)nb * sizeof(double), hipMemcpyDeviceToHost, st));
    RBF_HIP(hipMemcpyAsync(S->hred + kMaxNR * kMaxBlocks, K.bb, sizeof(double), hipMemcpyDeviceToHost, st));
    RBF_HIP(hipStreamSynchronize(st));
    double rr = 0.0;
    for (int bidx = 0; bidx < nb; ++bidx) rr += S->hred[bidx];
    const double bb = S->hred[kMaxNR * kMaxBlocks];
    const int f = S->hflag[0];
    const int iters = (f == 1) ? S->hflag[1] : it;
    if (stats) {
        stats->iterations = iters;
        stats->converged = (f == 1);
        stats->rel_residual = (bb > 0.0) ? std::sqrt(rr / bb) : std::sqrt(rr);
        stats->restarts = restarts;
        stats->final_flag = f;
    }
    if (f == -1) {
        rbf::set_error("preconditioned BiCGSTAB: non-finite value (iteration %d)", it);
        rc = RBF_E_NAN;
    } else if (f == 0 || f == 2) {
        rbf::set_error("preconditioned BiCGSTAB: no convergence (%d of %d iterations, %d restarts, flag %d)",
                       it, maxit, restarts, f);
        rc = RBF_E_NOCONV;
    }
    last_iters = iters;
    if (f == 1) {
        S->p_hist[S->p_pos] = iters;
        S->p_pos = (S->p_pos + 1) % 3;
        S->p_nhist = std::min(3, S->p_nhist + 1);
    }
    return rc;
}

// Viscous solve by Jacobi sweeps (see k_h_jac); same contract as hbicgstab.
rbf_status hjacobi(rbf_solver *S, EllM A, const double *b, double *x, double tol, int maxit,
                   int &last_iters, rbf_solve_stats *stats) {
    hipStream_t st = S->st;
    JKry J = S->jk;
    J.x0 = x;
    const int64_t n = A.n;
    const int nb = nblocks_rows(n);
    const dim3 grid(nb), block(kThreads);
    const double tol2 = tol * tol;
    const bool k28 = A.k == 28;
    RBF_HIP(hipMemsetAsync(J.flag, 0, 2 * sizeof(int), st));
    // Sweep i tests x_{i-1}; x_maxit is tested by sweep maxit + 1.
    int it = 0, f = 0;
    int batch = std::max(2, last_iters + 2);
    for (;;) {
        const int stop = std::min(maxit + 2, it + batch);
        for (; it < stop; ++it) {
            if (it == 0) {
                if (k28) hipLaunchKernelGGL((k_h_jac2<true>), grid, dim3(2 * kThreads), 0, st, A, b, J, it, tol2);
                else hipLaunchKernelGGL((k_h_jac<0, true>), grid, block, 0, st, A, b, J, it, tol2);
            } else {
                if (k28) hipLaunchKernelGGL((k_h_jac2<false>), grid, dim3(2 * kThreads), 0, st, A, b, J, it, tol2);
                else hipLaunchKernelGGL((k_h_jac<0, false>), grid, block, 0, st, A, b, J, it, tol2);
            }
        }
        RBF_CHECK_LAUNCH();
        RBF_HIP(hipMemcpyAsync(S->hflag, J.flag, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
        RBF_HIP(hipStreamSynchronize(st));
        f = S->hflag[0];
        if (f != 0 || it >= maxit + 2) break;
        batch = 2;
    }
    // The accepted iterate, or the newest one when the sweeps ran out.
    const int fin = (f != 0) ? S->hflag[1] : it;
    if (fin > 0)  // iterate fin lives in J.x[fin & 1], interleaved
        hipLaunchKernelGGL(k_h_deint, dim3(rbf::blocks_for(n, 256)), dim3(256), 0, st, n,
                           reinterpret_cast<const double2 *>(J.x[fin & 1]), x);
    // Statistics: the sweep that produced the accepted iterate's test left
    // the partials of its true residual and of ||b||^2 (slot fin & 1); after
    // running out of sweeps the newest iterate's residual is recomputed.
    const double *pf = J.part + (int64_t)(fin & 1) * 2 * kHR * kMaxBlocks;
    if (f != 1) {
        if (k28) hipLaunchKernelGGL((k_resid<kHR, 28>), grid, block, 0, st, A, b, x, S->rpart, nullptr);
        else hipLaunchKernelGGL((k_resid<kHR, 0>), grid, block, 0, st, A, b, x, S->rpart, nullptr);
        RBF_CHECK_LAUNCH();
        RBF_HIP(hipMemcpyAsync(S->hred, S->rpart, (size_t)kHR * nb * sizeof(double), hipMemcpyDeviceToHost, st));
    } else {
        for (int c = 0; c < kHR; ++c)
            RBF_HIP(hipMemcpyAsync(S->hred + c * nb, pf + (int64_t)c * kMaxBlocks, nb * sizeof(double),
                                   hipMemcpyDeviceToHost, st));
    }
    // ||b||^2 partials (b is fixed): from the same sweep, or from the last
    // sweep launched when none was accepted (every launched sweep ran).
    const double *pb = ((f == 1) ? pf : J.part + (int64_t)((std::max(it, 1) - 1) & 1) * 2 * kHR * kMaxBlocks) +
                       (int64_t)kHR * kMaxBlocks;
    for (int c = 0; c < kHR; ++c)
        RBF_HIP(hipMemcpyAsync(S->hred + kMaxNR * nb + c * nb, pb + (int64_t)c * kMaxBlocks,
                               nb * sizeof(double), hipMemcpyDeviceToHost, st));
    RBF_HIP(hipStreamSynchronize(st));
    rbf_status rc = RBF_OK;
    for (int c = 0; c < kHR; ++c) {
        double rr = 0.0, bb = 0.0;
        for (int bidx = 0; bidx < nb; ++bidx) {
            rr += S->hred[c * nb + bidx];
            bb += S->hred[kMaxNR * nb + c * nb + bidx];
        }
        if (stats) {
            stats[c].iterations = fin;
            stats[c].converged = (f == 1);
            stats[c].rel_residual = (bb > 0.0) ? std::sqrt(rr / bb) : std::sqrt(rr);
            stats[c].restarts = 0;
            stats[c].final_flag = f;
        }
    }
    if (f == -1) {
        rbf::set_error("Jacobi sweeps: non-finite residual (sweep %d)", fin);
        rc = RBF_E_NAN;
    } else if (f != 1) {
        rbf::set_error("Jacobi sweeps: no convergence (%d of %d sweeps)", it, maxit);
        rc = RBF_E_NOCONV;
    }
    last_iters = fin;
    return rc;
}

// Mixed-precision viscous solve (see k_hm_res): outer FP64 residuals with
// FP32 sweeps between them; same contract as hjacobi, with iterations
// counting outer refinement steps.
rbf_status hmixed(rbf_solver *S, EllM A, const double *b, double *x, double tol, int maxit,
                  int &last_iters, rbf_solve_stats *stats) {
    hipStream_t st = S->st;
    HMix X = S->hm;
    const int64_t n = A.n;
    const int nb = nblocks_rows(n);
    const dim3 grid(nb), block(kThreads);
    const double tol2 = tol * tol;
    const bool k28 = A.k == 28;
    hipLaunchKernelGGL(k_hm_clear, dim3(1), dim3(64), 0, st, X.flag);
    auto sweeps = [&](int i) {
        for (int s = 0; s < kHMixSweeps; ++s) {
            const bool test = s == 0, last = s == kHMixSweeps - 1;
#define HM_SWEEP(KT, T, L) hipLaunchKernelGGL((k_hm_sweep<KT, T, L>), grid, block, 0, st, X, i, s, tol2, nb)
            if (k28) {
                if (test && last) HM_SWEEP(28, true, true);
                else if (test) HM_SWEEP(28, true, false);
                else if (last) HM_SWEEP(28, false, true);
                else HM_SWEEP(28, false, false);
            } else {
                if (test && last) HM_SWEEP(0, true, true);
                else if (test) HM_SWEEP(0, true, false);
                else if (last) HM_SWEEP(0, false, true);
                else HM_SWEEP(0, false, false);
            }
#undef HM_SWEEP
        }
    };
    // Outer iteration i launches r_i (tested by the sweep after it) and its
    // sweeps; iteration maxit only tests.
    int i = 0, f = 0;
    int batch = std::max(1, last_iters + 1);
    for (;;) {
        const int stop = std::min(maxit + 1, i + batch);
        for (; i < stop; ++i) {
            if (i == 0) {
                if (k28) hipLaunchKernelGGL((k_hm_res<28, true>), grid, block, 0, st, A, b, x, X, i);
                else hipLaunchKernelGGL((k_hm_res<0, true>), grid, block, 0, st, A, b, x, X, i);
            } else {
                if (k28) hipLaunchKernelGGL((k_hm_res<28, false>), grid, block, 0, st, A, b, x, X, i);
                else hipLaunchKernelGGL((k_hm_res<0, false>), grid, block, 0, st, A, b, x, X, i);
            }
            sweeps(i);
        }
        RBF_CHECK_LAUNCH();
        RBF_HIP(hipMemcpyAsync(S->hflag, X.flag, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
        RBF_HIP(hipStreamSynchronize(st));
        f = S->hflag[0];
        if (f != 0 || i > maxit) break;
        batch = 1;
    }
    // The iterate X.x is x_fin when accepted (the sweeps after the test exit).
    const int fin = (f != 0) ? S->hflag[1] : maxit;
    hipLaunchKernelGGL(k_h_deint, dim3(rbf::blocks_for(n, 256)), dim3(256), 0, st, n, X.x, x);
    RBF_CHECK_LAUNCH();
    const double *pf = X.part + (int64_t)(fin & 1) * 2 * kHR * kMaxBlocks;
    for (int c = 0; c < 2 * kHR; ++c)
        RBF_HIP(hipMemcpyAsync(S->hred + c * nb, pf + (int64_t)c * kMaxBlocks, nb * sizeof(double),
                               hipMemcpyDeviceToHost, st));
    RBF_HIP(hipStreamSynchronize(st));
    rbf_status rc = RBF_OK;
    for (int c = 0; c < kHR; ++c) {
        double rr = 0.0, bb = 0.0;
        for (int bidx = 0; bidx < nb; ++bidx) {
            rr += S->hred[c * nb + bidx];
            bb += S->hred[(kHR + c) * nb + bidx];
        }
        if (stats) {
            stats[c].iterations = fin;
            stats[c].converged = (f == 1);
            stats[c].rel_residual = (bb > 0.0) ? std::sqrt(rr / bb) : std::sqrt(rr);
            stats[c].restarts = 0;
            stats[c].final_flag = f;
        }
    }
    if (f == -1) {
        rbf::set_error("mixed-precision viscous solve: non-finite residual (outer step %d)", fin);
        rc = RBF_E_NAN;
    } else if (f != 1) {
        rbf::set_error("mixed-precision viscous solve: no convergence (%d outer steps)", maxit);
        rc = RBF_E_NOCONV;
    }
    last_iters = fin;
    return rc;
}

// Viscous solve (both components): Jacobi right-preconditioned BiCGSTAB
// with explicit preconditioned directions; same contract as
// bicgstab<2, true> for a matrix without the rank-one border (A.u1 unset).
// Per iteration: k_h_dir, k_h_av (v), k_h_s, k_h_av (t).
rbf_status hbicgstab(rbf_solver *S, EllM A, const double *b, double *x, double tol, int maxit,
                     int &last_iters, rbf_solve_stats *stats) {
    hipStream_t st = S->st;
    HKry &K = S->hk;
    const int64_t n = A.n;
    const int nb = nblocks_rows(n);
    const dim3 grid(nb), block(kThreads);
    const double tol2 = tol * tol;
    const bool k28 = A.k == 28;
    auto init = [&]() {
        if (k28) hipLaunchKernelGGL((k_h_init<28>), grid, block, 0, st, A, b, x, K);
        else hipLaunchKernelGGL((k_h_init<0>), grid, block, 0, st, A, b, x, K);
    };
    auto av = [&](int mode, const double *y, double *out) {
        if (k28) {
            if (mode == 0) hipLaunchKernelGGL((k_h_av<28, 0>), grid, block, 0, st, A, K, y, out);
            else hipLaunchKernelGGL((k_h_av<28, 1>), grid, block, 0, st, A, K, y, out);
        } else {
            if (mode == 0) hipLaunchKernelGGL((k_h_av<0, 0>), grid, block, 0, st, A, K, y, out);
            else hipLaunchKernelGGL((k_h_av<0, 1>), grid, block, 0, st, A, K, y, out);
        }
    };
    init();
    int it = 0, i0 = 0, restarts = 0;
    rbf_status rc = RBF_OK;
    int batch = std::max(2, last_iters > 0 ? last_iters : 4);
    int win = kStall;
    bool done = false;
    while (!done) {
        const int stop = std::min(maxit + 1, it + batch);
        for (; it < stop; ++it) {
            hipLaunchKernelGGL(k_h_dir, grid, block, 0, st, K, A.dinv, x, n, it, i0);
            av(0, K.ph, K.v);
            hipLaunchKernelGGL(k_h_s, grid, block, 0, st, K, A.dinv, n, it, i0, tol2, win);
            av(1, K.sh, K.t);
        }
        RBF_CHECK_LAUNCH();
        RBF_HIP(hipMemcpyAsync(S->hflag, K.flag, kHR * sizeof(int), hipMemcpyDeviceToHost, st));
        RBF_HIP(hipMemcpyAsync(S->hflag + kMaxNR, K.iters, kHR * sizeof(int), hipMemcpyDeviceToHost, st));
        RBF_HIP(hipStreamSynchronize(st));
        prof_flush(S);
        done = true;
        bool restart = false;
        int brk_at = it;
        for (int c = 0; c < kHR; ++c) {
            if (S->hflag[c] == 0) done = false;
            if (S->hflag[c] == 2) {
                restart = true;
                brk_at = std::min(brk_at, S->hflag[kMaxNR + c]);
            }
        }
        if (restart && it <= maxit && restarts < 50) {
            ++restarts;
            it = i0 = brk_at;
            init();
            done = false;
            win = std::min(2 * win, 1 << 20);
            continue;
        }
        if (!done && it > maxit) break;
        batch = 2;
    }
    if (k28) hipLaunchKernelGGL((k_resid<kHR, 28>), grid, block, 0, st, A, b, x, S->rpart, nullptr);
    else hipLaunchKernelGGL((k_resid<kHR, 0>), grid, block, 0, st, A, b, x, S->rpart, nullptr);
    RBF_CHECK_LAUNCH();
    RBF_HIP(hipMemcpyAsync(S->hred, S->rpart, (size_t)kHR * nb * sizeof(double), hipMemcpyDeviceToHost, st));
    RBF_HIP(hipMemcpyAsync(S->hred + kMaxNR * kMaxBlocks, K.bb, kHR * sizeof(double), hipMemcpyDeviceToHost, st));
    RBF_HIP(hipStreamSynchronize(st));
    int maxi = 0;
    for (int c = 0; c < kHR; ++c) {
        double rr = 0.0;
        for (int bidx = 0; bidx < nb; ++bidx) rr += S->hred[c * nb + bidx];
        const double bb = S->hred[kMaxNR * kMaxBlocks + c];
        const int f = S->hflag[c];
        const int iters = (f == 1) ? S->hflag[kMaxNR + c] : it;
        maxi = std::max(maxi, iters);
        if (stats) {
            stats[c].iterations = iters;
            stats[c].converged = (f == 1);
            stats[c].rel_residual = (bb > 0.0) ? std::sqrt(rr / bb) : std::sqrt(rr);
            stats[c].restarts = restarts;
            stats[c].final_flag = f;
        }
        if (f == -1) {
            rbf::set_error("BiCGSTAB: non-finite value (rhs %d, iteration %d)", c, it);
            rc = RBF_E_NAN;
        } else if ((f == 0 || f == 2) && rc == RBF_OK) {
            rbf::set_error("BiCGSTAB: no convergence (rhs %d, %d of %d iterations, %d restarts, flag %d)",
                           c, it, maxit, restarts, f);
            rc = RBF_E_NOCONV;
        }
    }
    last_iters = maxi;
    return rc;
}

// Pressure solve on the row-scaled bordered system (x: guess in, solution out).
rbf_status aux_solve(rbf_solver *S, EllM A, const double *b, double *x, rbf_solve_stats *stats);

rbf_status poisson_solve(rbf_solver *S, const double *b, double *x, rbf_solve_stats *stats) {
    EllM P{S->idx_pp, S->p_w, nullptr, S->M, S->k, S->p_u1, S->p_vscale};
    if (S->aux_on) return aux_solve(S, P, b, x, stats);
    if (S->pc_on) return pbicgstab(S, P, b, x, S->rtol_p, S->maxit_p, S->last_iters_p, stats);
    return bicgstab<1, false>(S, S->kp, P, b, x, S->rtol_p, S->maxit_p, S->last_iters_p, stats);
}

// DCT-II eigenbasis of the 1-D Neumann second difference on n points
// (tridiag(1, -2, 1) with -1 at both ends): q_k(a) = cos(pi k (a + 1/2) / n),
// lam_k = -4 sin^2(pi k / (2 n)).  Q(a, k) at Q[a + k n]; Q^-1(k, a) =
// d_k Q(a, k) with d_0 = 1/n, d_k = 2/n, at Qi[k + a n].
void dct2_basis(int n, std::vector<double> &Q, std::vector<double> &Qi, std::vector<double> &lam) {
    Q.assign((size_t)n * n, 0.0);
    Qi.assign((size_t)n * n, 0.0);
    lam.assign(n, 0.0);
    const double pi = 3.14159265358979323846;
    for (int k = 0; k < n; ++k) {
        const double sk = std::sin(pi * k / (2.0 * n));
        lam[k] = -4.0 * sk * sk;
        for (int a = 0; a < n; ++a) {
            const int64_t mth = ((int64_t)k * (2 * a + 1)) % (4LL * n);  // angle pi mth / (2n)
            const double c = std::cos(pi * (double)mth / (2.0 * n));
            Q[(size_t)a + (size_t)k * n] = c;
            Qi[(size_t)k + (size_t)a * n] = (k == 0 ? 1.0 / n : 2.0 / n) * c;
        }
    }
}

// True if the P-nodes are the jittered (K+1)^2 lattice the preconditioner
// assumes: row-major vertices within half a spacing of (i h, j h), wall
// nodes exactly on their walls and tagged, interior nodes untagged.
bool is_lattice(const std::vector<double> &xp, const std::vector<int8_t> &tag, int64_t m, int &Kout) {
    const int64_t K1 = (int64_t)std::llround(std::sqrt((double)m));
    if (K1 * K1 != m || K1 < 5) return false;
    const int K = (int)(K1 - 1);
    const double h = 1.0 / K;
    for (int64_t v = 0; v < m; ++v) {
        const int i = (int)(v % K1), j = (int)(v / K1);
        const double x = xp[v], y = xp[m + v];
        const bool bnd = (i == 0 || i == K || j == 0 || j == K);
        if (bnd != (tag[v] != 0)) return false;
        if (!(std::fabs(x - i * h) < 0.5 * h && std::fabs(y - j * h) < 0.5 * h)) return false;
        if ((i == 0 && x != 0.0) || (i == K && x != 1.0) || (j == 0 && y != 0.0) ||
            (j == K && y != 1.0))
            return false;
    }
    Kout = K;
    return true;
}

// Set up the lattice preconditioner if the grid allows it (mode: RBF_PRECOND_*).
rbf_status setup_lattice_pc(rbf_solver *S, const rbf_grid *g, int mode) {
    if (mode == RBF_PRECOND_NONE || mode == RBF_PRECOND_AUX) return RBF_OK;
    const int64_t M = S->M;
    hipStream_t st = S->st;
    std::vector<double> hx(2 * M);
    std::vector<int8_t> ht(M);
    RBF_HIP(hipMemcpyAsync(hx.data(), g->xp, 2 * M * sizeof(double), hipMemcpyDeviceToHost, st));
    RBF_HIP(hipMemcpyAsync(ht.data(), g->p_tag, M, hipMemcpyDeviceToHost, st));
    RBF_HIP(hipStreamSynchronize(st));
    int K = 0;
    if (!is_lattice(hx, ht, M, K)) {
        RBF_ARG(mode != RBF_PRECOND_LATTICE,
                "rbf_solver_create: RBF_PRECOND_LATTICE needs the P-nodes on a jittered "
                "(K+1)^2 lattice of the unit square (row-major, walls tagged)");
        return RBF_OK;
    }
    if (K - 1 > 64 * kTriChunk) {  // the tridiagonal kernel holds one mode per wavefront
        RBF_ARG(mode != RBF_PRECOND_LATTICE,
                "rbf_solver_create: RBF_PRECOND_LATTICE supports K <= %d (got K = %d)",
                64 * kTriChunk + 1, K);
        return RBF_OK;
    }
    const int n = K - 1;
    std::vector<double> Q, Qi, lam;
    dct2_basis(n, Q, Qi, lam);
    std::vector<int> cell(M);
    std::vector<double> fx(M), fy(M);
    for (int64_t v = 0; v < M; ++v) {
        const double sx = hx[v] * K, sy = hx[M + v] * K;
        const int i0 = std::min(std::max((int)std::floor(sx), 0), K - 1);
        const int j0 = std::min(std::max((int)std::floor(sy), 0), K - 1);
        cell[v] = j0 * (K + 1) + i0;
        fx[v] = std::min(std::max(sx - i0, 0.0), 1.0);
        fy[v] = std::min(std::max(sy - j0, 0.0), 1.0);
    }
    // V = Q^T w for the boundary-count weights w(a, b) = [a = 0] + [a = n-1]
    // + [b = 0] + [b = n-1] + [corner]: with s_k = sum_a Q(a, k) and
    // e_k = Q(0, k) + Q(n-1, k), V(k, b) = e_k + (s_k + e_k) ([b = 0] + [b = n-1]).
    std::vector<double> V((size_t)n * n);
    for (int k = 0; k < n; ++k) {
        double sk = 0.0;
        for (int a = 0; a < n; ++a) sk += Q[(size_t)a + (size_t)k * n];
        const double ek = Q[(size_t)k * n] + Q[(size_t)(n - 1) + (size_t)k * n];
        for (int b = 0; b < n; ++b)
            V[(size_t)k * n + b] = ek + ((b == 0 || b == n - 1) ? sk + ek : 0.0);
    }
    const size_t nn = (size_t)n * n;
    const int nt = (n + 15) / 16;
    Lat &L = S->lat;
    L.ntiles = nt * nt;
    L.f32 = S->mixed ? 1 : 0;
    const size_t es = L.f32 ? sizeof(float) : sizeof(double);
    int *dcell;
    double *dfx, *dfy, *dlam, *dV;
    void *dQ, *dQi;
    ALLOC(dcell, M);
    ALLOC(dfx, M);
    ALLOC(dfy, M);
    ALLOC(dlam, n);
    ALLOC(dV, nn);
    rbf_status rc;
    for (void **a : {&dQ, &dQi, &L.X, &L.T, &L.W})
        if ((rc = dalloc(S, a, nn * es)) != RBF_OK) return rc;
    ALLOC(L.mean, 1);
    ALLOC(L.partW, n);
    PKry &P = S->pk;
    for (double **q : {&P.r, &P.rh, &P.p[0], &P.p[1], &P.v, &P.s, &P.t, &P.ph, &P.sh}) ALLOC(*q, M);
    ALLOC(P.partI, 2 * kMaxBlocks);
    ALLOC(P.part1, 2 * kMaxBlocks);
    ALLOC(P.partGs, kMaxBlocks);
    ALLOC(P.part3, kMaxBlocks);
    ALLOC(P.part6, 3 * kMaxBlocks);
    ALLOC(P.partS, kMaxBlocks);
    ALLOC(P.rec, (int64_t)(S->maxit_p + 2) * 4);
    ALLOC(P.bb, 1);
    ALLOC(P.rhrh, 1);
    ALLOC(P.best, 4);
    ALLOC(P.flag, 8);  // flag, iters, 3 status doubles (see PKry)
    P.iters = P.flag + 1;
    P.stat = reinterpret_cast<double *>(P.flag + 2);
    RBF_HIP(hipMemcpyAsync(dcell, cell.data(), M * sizeof(int), hipMemcpyHostToDevice, st));
    RBF_HIP(hipMemcpyAsync(dfx, fx.data(), M * sizeof(double), hipMemcpyHostToDevice, st));
    RBF_HIP(hipMemcpyAsync(dfy, fy.data(), M * sizeof(double), hipMemcpyHostToDevice, st));
    RBF_HIP(hipMemcpyAsync(dlam, lam.data(), n * sizeof(double), hipMemcpyHostToDevice, st));
    RBF_HIP(hipMemcpyAsync(dV, V.data(), nn * sizeof(double), hipMemcpyHostToDevice, st));
    std::vector<float> Qf, Qif;
    const void *hQ = Q.data(), *hQi = Qi.data();
    if (L.f32) {  // transform matrices rounded to FP32
        Qf.assign(Q.begin(), Q.end());
        Qif.assign(Qi.begin(), Qi.end());
        hQ = Qf.data();
        hQi = Qif.data();
    }
    RBF_HIP(hipMemcpyAsync(dQ, hQ, nn * es, hipMemcpyHostToDevice, st));
    RBF_HIP(hipMemcpyAsync(dQi, hQi, nn * es, hipMemcpyHostToDevice, st));
    RBF_HIP(hipMemsetAsync(L.X, 0, nn * es, st));
    RBF_HIP(hipMemsetAsync(P.flag, 0, sizeof(int), st));
    RBF_HIP(hipStreamSynchronize(st));
    L.K = K;
    L.n = n;
    L.h = 1.0 / K;
    L.c = S->p_vscale;
    L.rs = S->p_rowscale;
    L.cell = dcell;
    L.fx = dfx;
    L.fy = dfy;
    L.Q = dQ;
    L.Qi = dQi;
    L.lam = dlam;
    L.V = dV;
    L.flag = P.flag;
    S->pc_on = true;
    return RBF_OK;
}

template <class F>
void launch_kt(int k, F f) {
    if (k == 28) f(std::integral_constant<int, 28>{});
    else f(std::integral_constant<int, 0>{});
}

rbf_status copy_in(rbf_solver *S, void *dst, const void *src, size_t bytes) {
    RBF_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, S->st));
    return RBF_OK;
}

// ------------------------------------- auxiliary-lattice pressure path --
// One application z = B^-1 (ys y) of the two-level preconditioner
// (pressure_aux.h): smoother, residual, restriction, lattice transform
// solve, interpolation, smoother.
template <class T>
void aux_apply(rbf_solver *S, const AuxOps<T> &P, FgDev<T> &F, const T *y, const T *yd,
               const double *ys, T *z, bool sample = false) {
    hipStream_t st = S->st;
    const dim3 grid(nblocks_rows(P.m)), block(kThreads);
    const int nq = S->lat.n * S->lat.n;
    // Pre-smoothing: x1 = W y (implicit, yd), further sweeps into F.x1.
    const T *u = yd;
    const double *us = ys;
    static_assert(kAuxSweeps == 1 || kAuxSweeps == 2, "one or two smoothing sweeps");
    if constexpr (kAuxSweeps == 2) {
        launch_kt(P.k, [&](auto KT) {
            hipLaunchKernelGGL((k_aux_pre<decltype(KT)::value, T>),
                               aux_grid<decltype(KT)::value>(P.m, grid.x), block, 0, st, P, y, yd, ys,
                               F.x1, F.s.flag);
        });
        u = F.x1;
        us = F.s.one;
    }
    launch_kt(P.k, [&](auto KT) {
        hipLaunchKernelGGL((k_aux_res<decltype(KT)::value, T>),
                           aux_grid<decltype(KT)::value>(P.m, grid.x), block, 0, st, P, y, ys, u,
                           us, F.res, F.s.flag);
    });
    hipLaunchKernelGGL(k_aux_restrict<T>, dim3(rbf::blocks_for(4 * (int64_t)nq, 256)), dim3(256), 0,
                       st, P, S->lat, F.res, nq);
    pc_apply(S, sample);
    hipLaunchKernelGGL(k_aux_interp<T>, grid, block, 0, st, P, S->lat, u, us, F.t1, F.s.partZ);
    // Post-smoothing: the first sweep adds the border's constant.
    T *zin = F.t1;
    if constexpr (kAuxSweeps == 2) {
        if (P.k == 28)
            hipLaunchKernelGGL((k_aux_post2<T, true>), grid, dim3(2 * kThreads), 0, st, P, S->lat, y,
                               ys, F.t1, F.s.partZ, F.z1, F.s.partO);
        else
            hipLaunchKernelGGL((k_aux_post<0, T, true>), grid, block, 0, st, P, S->lat, y, ys, F.t1,
                               F.s.partZ, F.z1, F.s.partO);
        zin = F.z1;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (sample) prof_pair(S, RBF_PROF_SMOOTH, e0, e1);
    if (P.k == 28)
        hipExtLaunchKernelGGL((k_aux_post2<T, kAuxSweeps == 1>), grid, dim3(2 * kThreads), 0, st, e0,
                              e1, 0, P, S->lat, y, ys, zin, F.s.partZ, z, F.s.partO);
    else
        hipExtLaunchKernelGGL((k_aux_post<0, T, kAuxSweeps == 1>), grid, block, 0, st, e0, e1, 0, P,
                              S->lat, y, ys, zin, F.s.partZ, z, F.s.partO);
}

// Orthogonalisation of the Arnoldi vectors: classical Gram-Schmidt once
// (h2 stays zero), or applied twice when true.  One pass takes the same
// number of steps to the same true residual on the h = 1/400 cavity and the
// cylinder (32.3 and 35.2 per time step) and saves a reduction and a pass
// over the basis per step; convergence is only declared from the true
// residual recomputed at a restart, so a loss of orthogonality can cost
// steps but not accuracy.
constexpr bool kFgReorth = false;

// Flexible GMRES(kFgMax) on the pressure system with the two-level
// preconditioner (x: guess in, solution out).  Every cycle starts from the
// FP64 residual; with T = float the cycle is one step of iterative
// refinement (see pressure_aux.h).  maxit counts Arnoldi steps
// (preconditioner applications).
template <class T>
rbf_status fgmres_run(rbf_solver *S, const AuxOps<T> &P, FgDev<T> &F, EllM A, const double *b,
                      double *x, double tol, int maxit, int &last_iters, rbf_solve_stats *stats) {
    hipStream_t st = S->st;
    const int64_t m = A.n;
    const int nb = nblocks_rows(m);
    const dim3 grid(nb), block(kThreads), one(1), red(256);
    const int mr = kFgMax;
    const int mixed = std::is_same<T, float>::value ? 1 : 0;
    FgScal &Fs = F.s;
    S->lat.flag = Fs.flag;  // the transform stages exit with the Krylov flag
    int total = 0, cycles = 0, f = 0;
    bool first = true;
    // Expected steps of the first cycle: the last solve's count (warm starts
    // of consecutive steps need about as many).
    int expect = S->p_nhist ? S->p_hist[(S->p_pos + 2) % 3] : 0;
    auto status = [&]() -> rbf_status {
        RBF_HIP(hipMemcpyAsync(S->hflag, Fs.flag, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
        RBF_HIP(hipMemcpyAsync(S->hflag + 2, Fs.stat, 5 * sizeof(double), hipMemcpyDeviceToHost, st));
        RBF_HIP(hipStreamSynchronize(st));
        prof_flush(S, S->hflag[1]);
        return RBF_OK;
    };
    rbf_status rc = RBF_OK;
    for (;;) {
        if (A.u1) hipLaunchKernelGGL((k_sum<1>), grid, block, 0, st, m, x, S->kp.partX);
        launch_kt(A.k, [&](auto KT) {
            hipLaunchKernelGGL((k_fg_init<decltype(KT)::value, T>), grid, block, 0, st, A, b, x,
                               S->kp.partX, F.V, P.dinv, F.wd, Fs.part);
        });
        hipLaunchKernelGGL(k_fg_reduce<false>, dim3(2), red, 0, st, Fs.part, nb, 2, Fs.h1, Fs.flag);
        hipLaunchKernelGGL(k_fg_start, one, one, 0, st, Fs, Fs.h1, tol, mixed, first ? 1 : 0);
        first = false;
        if (total >= maxit) {  // only the convergence test of the iterate
            if ((rc = status()) != RBF_OK) return rc;
            f = S->hflag[0];
            break;
        }
        int j = 0;
        // First batch of a cycle: the steps the last solve needed beyond
        // those already taken, less one (later batches follow the
        // residual's rate); 6 when nothing is known.
        int batch = 6;
        if (expect > 0)
            batch = (cycles == 0) ? std::max(2, std::min(mr, expect - 2))
                                  : std::max(2, std::min(6, expect - total - 1));
        for (;;) {
            const int stop = std::min(mr, j + batch);
            for (; j < stop; ++j) {
                const int64_t o = (int64_t)j * m;
                const bool sample = S->prof_every > 0 && (S->prof_launches++ % S->prof_every) == 0;
                S->prof_tag_now = j;
                aux_apply(S, P, F, F.V + o, F.wd, Fs.vs + j, F.Z + o, sample);
                hipEvent_t e0 = nullptr, e1 = nullptr, g0 = nullptr, g1 = nullptr;
                if (sample) {
                    prof_pair(S, RBF_PROF_SPMV, e0, e1);
                    prof_pair(S, RBF_PROF_GS, g0, g1);
                }
                if (P.k == 28)
                    hipExtLaunchKernelGGL((k_fg_av2<T>), grid, dim3(kAvThreads), 0, st, e0, e1, 0, P,
                                          A.u1, A.vscale, F, j);
                else
                    hipExtLaunchKernelGGL((k_fg_av<0, T>), grid, block, 0, st, e0, e1, 0, P, A.u1,
                                          A.vscale, F, j);
                hipLaunchKernelGGL(k_fg_reduce<true>, dim3(j + 1), red, 0, st, Fs.part, nb, j + 1,
                                   Fs.h1, Fs.flag);
                if constexpr (kFgReorth) {
                    hipExtLaunchKernelGGL((k_fg_gs<T, 1>), grid, dim3(2 * kThreads), 0, st, g0, g1, 0,
                                          F, Fs.h1, P.dinv, m, j);
                    hipLaunchKernelGGL(k_fg_reduce<true>, dim3(j + 1), red, 0, st, Fs.part, nb, j + 1,
                                       Fs.h2, Fs.flag);
                    hipLaunchKernelGGL((k_fg_gs<T, 2>), grid, dim3(2 * kThreads), 0, st, F, Fs.h2,
                                       P.dinv, m, j);
                } else {
                    hipExtLaunchKernelGGL((k_fg_gs<T, 2>), grid, dim3(2 * kThreads), 0, st, g0, g1, 0,
                                          F, Fs.h1, P.dinv, m, j);
                }
                hipLaunchKernelGGL(k_fg_tail, one, red, 0, st, Fs, j, mr, nb);
                S->prof_tag_now = -1;
            }
            RBF_CHECK_LAUNCH();
            if ((rc = status()) != RBF_OK) return rc;
            f = S->hflag[0];
            if (f != 0 || j >= mr) break;
            // Next batch from the residual's rate over the last four steps.
            const double *hs = reinterpret_cast<const double *>(S->hflag + 2);
            batch = 4;
            if (hs[0] > 0.0 && hs[1] > hs[0] && hs[2] > 0.0) {
                const double rate = std::log(hs[0] / hs[1]) / 4.0;
                const double need = std::log(hs[2] / hs[0]) / rate;
                if (std::isfinite(need)) batch = std::max(1, std::min(12, (int)std::ceil(need)));
            }
        }
        const int nstep = S->hflag[1];
        total += nstep;
        if (f == 1 || f == -1) break;
        if (nstep <= 0) {  // no step was taken: nothing would change
            f = 0;
            break;
        }
        hipLaunchKernelGGL(k_fg_solve, one, red, 0, st, Fs, nstep, mr);
        hipLaunchKernelGGL((k_fg_x<T>), grid, block, 0, st, F.Z, Fs.y, nstep, m, x);
        ++cycles;
    }
    const double *hs = reinterpret_cast<const double *>(S->hflag + 2);
    const double bb = hs[3], beta = hs[4];
    if (stats) {
        stats->iterations = total;
        stats->converged = (f == 1);
        stats->rel_residual = (bb > 0.0) ? beta / std::sqrt(bb) : beta;
        stats->restarts = cycles;
        stats->final_flag = f;
    }
    if (f == -1) {
        rbf::set_error("FGMRES: non-finite value (after %d steps)", total);
        rc = RBF_E_NAN;
    } else if (f != 1) {
        rbf::set_error("FGMRES: no convergence (%d of %d steps, %d cycles)", total, maxit, cycles);
        rc = RBF_E_NOCONV;
    }
    last_iters = total;
    if (f == 1) {
        S->p_hist[S->p_pos] = total;
        S->p_pos = (S->p_pos + 1) % 3;
        S->p_nhist = std::min(3, S->p_nhist + 1);
    }
    return rc;
}

rbf_status aux_solve(rbf_solver *S, EllM A, const double *b, double *x, rbf_solve_stats *stats) {
    A.vscale *= kAuxBorder;  // as S->lat.c
    if (S->mixed)
        return fgmres_run<float>(S, S->ax32, S->fg32, A, b, x, S->rtol_p, S->maxit_p,
                                 S->last_iters_p, stats);
    return fgmres_run<double>(S, S->ax64, S->fg64, A, b, x, S->rtol_p, S->maxit_p,
                              S->last_iters_p, stats);
}

template <class T>
rbf_status alloc_fg(rbf_solver *S, FgDev<T> &F, int64_t M) {
    const int mr = kFgMax;
    ALLOC(F.V, (int64_t)(mr + 1) * M);
    ALLOC(F.Z, (int64_t)mr * M);
    ALLOC(F.res, M);
    ALLOC(F.t1, M);
    ALLOC(F.wd, M);
    ALLOC(F.x1, M);
    ALLOC(F.z1, M);
    FgScal &s = F.s;
    ALLOC(s.vs, mr + 1);
    ALLOC(s.part, (int64_t)(kFgMax + 2) * kMaxBlocks);
    ALLOC(s.h1, mr + 1);
    ALLOC(s.h2, mr + 1);
    RBF_HIP(hipMemsetAsync(s.h2, 0, (mr + 1) * sizeof(double), S->st));
    ALLOC(s.hn2, 1);
    ALLOC(s.H, (int64_t)(mr + 1) * mr);
    ALLOC(s.cs, mr);
    ALLOC(s.sn, mr);
    ALLOC(s.g, mr + 1);
    ALLOC(s.y, mr);
    ALLOC(s.resh, mr + 1);
    ALLOC(s.partZ, kMaxBlocks);
    ALLOC(s.partO, kMaxBlocks);
    ALLOC(s.one, 1);
    const double unit = 1.0;
    RBF_HIP(hipMemcpyAsync(s.one, &unit, sizeof(double), hipMemcpyHostToDevice, S->st));
    ALLOC(s.flag, 16);  // flag, step, 5 status doubles (8-byte aligned at +2 ints)
    s.step = s.flag + 1;
    s.stat = reinterpret_cast<double *>(s.flag + 2);
    RBF_HIP(hipMemsetAsync(s.flag, 0, 16 * sizeof(int), S->st));
    return RBF_OK;
}

// Set up the two-level auxiliary-lattice preconditioner when the P-nodes'
// bounding box is a square (mode: RBF_PRECOND_*; AUTO uses it when the
// lattice preconditioner does not apply).
rbf_status setup_aux_pc(rbf_solver *S, const rbf_grid *g, int mode) {
    if (mode == RBF_PRECOND_NONE || mode == RBF_PRECOND_LATTICE || S->pc_on) return RBF_OK;
    const int64_t M = S->M;
    hipStream_t st = S->st;
    std::vector<double> hx(2 * M);
    std::vector<int8_t> ht(M);
    RBF_HIP(hipMemcpyAsync(hx.data(), g->xp, 2 * M * sizeof(double), hipMemcpyDeviceToHost, st));
    RBF_HIP(hipMemcpyAsync(ht.data(), g->p_tag, M, hipMemcpyDeviceToHost, st));
    RBF_HIP(hipStreamSynchronize(st));
    double x0 = INFINITY, x1 = -INFINITY, y0 = INFINITY, y1 = -INFINITY;
    for (int64_t v = 0; v < M; ++v) {
        x0 = std::min(x0, hx[v]);
        x1 = std::max(x1, hx[v]);
        y0 = std::min(y0, hx[M + v]);
        y1 = std::max(y1, hx[M + v]);
    }
    const double wx = x1 - x0, wy = y1 - y0;
    // Ka x Ka cells over the bounding box (cells of wx/Ka by wy/Ka; the
    // box's aspect ratio is limited so that the cells stay usable).
    const bool box_ok = wx > 0.0 && wy > 0.0 && wx <= 8.0 * wy && wy <= 8.0 * wx;
    // About one node spacing per lattice cell (M ~ 1.15 K^2 nodes on a
    // near-equilateral set of spacing 1/K: Ka ~ K).  A finer lattice makes
    // the coarse correction closer to the operator (on the h = 1/400 cavity
    // 39 FGMRES steps per time step instead of 52 with two spacings per
    // cell) for little more transform time while n stays within one pass of
    // k_pc_gemm (n <= 448).
    int Ka = (int)std::llround(0.95 * std::sqrt((double)M));
    Ka = std::max(4, std::min(Ka, 64 * kTriChunk + 1));
    if (!box_ok || M < 64) {
        RBF_ARG(mode != RBF_PRECOND_AUX,
                "rbf_solver_create: RBF_PRECOND_AUX needs P-nodes whose bounding box has sides within a factor 8 of each other");
        return RBF_OK;
    }
    const int n = Ka - 1, K1 = Ka + 1;
    const double hxa = wx / Ka, hya = wy / Ka;
    // Cells and bilinear coordinates of every node; restriction lists of the
    // interior lattice points from the interior nodes.
    std::vector<int> cell(M);
    std::vector<double> fx(M), fy(M);
    std::vector<int> cnt((size_t)n * n + 1, 0);
    auto corner_q = [&](int i, int j) { return (i >= 1 && i <= Ka - 1 && j >= 1 && j <= Ka - 1) ? (i - 1) * n + (j - 1) : -1; };
    for (int64_t v = 0; v < M; ++v) {
        const double sx = (hx[v] - x0) / hxa, sy = (hx[M + v] - y0) / hya;
        const int i0 = std::min(std::max((int)std::floor(sx), 0), Ka - 1);
        const int j0 = std::min(std::max((int)std::floor(sy), 0), Ka - 1);
        cell[v] = j0 * K1 + i0;
        fx[v] = std::min(std::max(sx - i0, 0.0), 1.0);
        fy[v] = std::min(std::max(sy - j0, 0.0), 1.0);
        if (ht[v] != 0) continue;
        for (int c = 0; c < 4; ++c) {
            const int q = corner_q(i0 + (c & 1), j0 + (c >> 1));
            if (q >= 0) ++cnt[q + 1];
        }
    }
    for (size_t q = 0; q < (size_t)n * n; ++q) cnt[q + 1] += cnt[q];
    std::vector<int> rptr(cnt), rcol(cnt.back());
    std::vector<double> rval(cnt.back()), wsum((size_t)n * n, 0.0);
    std::vector<int> fill(cnt.begin(), cnt.end() - 1);
    for (int64_t v = 0; v < M; ++v) {  // node order within each list
        if (ht[v] != 0) continue;
        const int i0 = cell[v] % K1, j0 = cell[v] / K1;
        for (int c = 0; c < 4; ++c) {
            const int q = corner_q(i0 + (c & 1), j0 + (c >> 1));
            if (q < 0) continue;
            const double wx = (c & 1) ? fx[v] : 1.0 - fx[v], wy = (c >> 1) ? fy[v] : 1.0 - fy[v];
            rcol[fill[q]] = (int)v;
            rval[fill[q]] = wx * wy;
            wsum[q] += wx * wy;
            ++fill[q];
        }
    }
    for (size_t q = 0; q < (size_t)n * n; ++q)
        for (int e = rptr[q]; e < rptr[q + 1]; ++e) rval[e] = (wsum[q] > 0.0) ? rval[e] / wsum[q] : 0.0;
    std::vector<double> Q, Qi, lam;
    dct2_basis(n, Q, Qi, lam);
    // Anisotropic cells: (T_x / hx^2 + T_y / hy^2) e = g becomes, per x-mode
    // k, (T_y + (hy/hx)^2 lam_k) w = hy^2 t.
    for (double &l : lam) l *= (hya / hxa) * (hya / hxa);
    const size_t nn = (size_t)n * n;
    const int nt = (n + 15) / 16;
    Lat &L = S->lat;
    L.ntiles = nt * nt;
    L.f32 = S->mixed ? 1 : 0;
    const size_t es = L.f32 ? sizeof(float) : sizeof(double);
    int *dcell, *drptr, *drcol;
    double *dfx, *dfy, *dlam, *dV, *drval;
    void *dQ, *dQi;
    ALLOC(dcell, M);
    ALLOC(dfx, M);
    ALLOC(dfy, M);
    ALLOC(dlam, n);
    ALLOC(dV, nn);
    ALLOC(drptr, nn + 1);
    ALLOC(drcol, std::max<size_t>(1, rcol.size()));
    ALLOC(drval, std::max<size_t>(1, rval.size()));
    rbf_status rc;
    for (void **a : {&dQ, &dQi, &L.X, &L.T, &L.W})
        if ((rc = dalloc(S, a, nn * es)) != RBF_OK) return rc;
    ALLOC(L.mean, 1);
    ALLOC(L.partW, n);
    RBF_HIP(hipMemcpyAsync(dcell, cell.data(), M * sizeof(int), hipMemcpyHostToDevice, st));
    RBF_HIP(hipMemcpyAsync(dfx, fx.data(), M * sizeof(double), hipMemcpyHostToDevice, st));
    RBF_HIP(hipMemcpyAsync(dfy, fy.data(), M * sizeof(double), hipMemcpyHostToDevice, st));
    RBF_HIP(hipMemcpyAsync(dlam, lam.data(), n * sizeof(double), hipMemcpyHostToDevice, st));
    RBF_HIP(hipMemsetAsync(dV, 0, nn * sizeof(double), st));
    RBF_HIP(hipMemcpyAsync(drptr, rptr.data(), (nn + 1) * sizeof(int), hipMemcpyHostToDevice, st));
    if (!rcol.empty()) {
        RBF_HIP(hipMemcpyAsync(drcol, rcol.data(), rcol.size() * sizeof(int), hipMemcpyHostToDevice, st));
        RBF_HIP(hipMemcpyAsync(drval, rval.data(), rval.size() * sizeof(double), hipMemcpyHostToDevice, st));
    }
    std::vector<float> Qf, Qif;
    const void *hQ = Q.data(), *hQi = Qi.data();
    if (L.f32) {
        Qf.assign(Q.begin(), Q.end());
        Qif.assign(Qi.begin(), Qi.end());
        hQ = Qf.data();
        hQi = Qif.data();
    }
    RBF_HIP(hipMemcpyAsync(dQ, hQ, nn * es, hipMemcpyHostToDevice, st));
    RBF_HIP(hipMemcpyAsync(dQi, hQi, nn * es, hipMemcpyHostToDevice, st));
    RBF_HIP(hipMemsetAsync(L.X, 0, nn * es, st));
    L.K = Ka;
    L.n = n;
    L.h = hya;
    L.c = S->p_vscale * kAuxBorder;  // the FGMRES operator's border scale
    L.rs = S->p_rowscale;
    L.cell = dcell;
    L.fx = dfx;
    L.fy = dfy;
    L.Q = dQ;
    L.Qi = dQi;
    L.lam = dlam;
    L.V = dV;
    // Row data of the smoother (FP64), and FP32 copies for mixed precision.
    double *ddinv, *dsinv;
    ALLOC(ddinv, M);
    ALLOC(dsinv, M);
    hipLaunchKernelGGL(k_aux_rows, dim3(rbf::blocks_for(M, 256)), dim3(256), 0, st, M, S->k,
                       S->p_w, S->p_rowscale, ddinv, dsinv);
    RBF_CHECK_LAUNCH();
    S->ax64 = AuxOps<double>{S->idx_pp, S->p_w, ddinv, dsinv, drptr, drcol, drval, M, S->k};
    // Weight of the second sweep of each smoothing pair, from the largest
    // eigenvalue nu of W A_s (power iteration): the pair's error polynomial
    // (1 - nu)(1 - w2 nu) stays within 1 in magnitude for w2 <= 1 / (nu - 1);
    // w2 is 0.85 of that bound, between 1 and 1.6, with nu raised by 5 %
    // (80 power steps approach it from below, within 5 % when the top
    // eigenvalues cluster).  The h = 1/400 cavity (nu = 1.47) gets about
    // 1.55: 32 instead of 35 FGMRES steps per time step; the graded
    // cylinder sets (nu = 1.74-1.88) stay near 1, where a fixed 1.5 made
    // their solves fail.
    {
        struct Scratch {
            double *x = nullptr, *y = nullptr, *part = nullptr;
            ~Scratch() {
                (void)hipFree(x);
                (void)hipFree(y);
                (void)hipFree(part);
            }
        } P;
        RBF_HIP(hipMalloc(&P.x, M * sizeof(double)));
        RBF_HIP(hipMalloc(&P.y, M * sizeof(double)));
        RBF_HIP(hipMalloc(&P.part, kMaxBlocks * sizeof(double)));
        const int nbp = nblocks_rows(M);
        std::vector<double> hp(nbp);
        hipLaunchKernelGGL(k_aux_power_start, dim3(rbf::blocks_for(M, 256)), dim3(256), 0, st, M, P.x);
        double scale = 1.0 / std::sqrt((double)M / 3.0), nu = 0.0;
        for (int it = 0; it < 80; ++it) {
            hipLaunchKernelGGL((k_aux_power<double>), dim3(nbp), dim3(kThreads), 0, st, S->ax64, P.x,
                               scale, P.y, P.part);
            RBF_CHECK_LAUNCH();
            RBF_HIP(hipMemcpyAsync(hp.data(), P.part, nbp * sizeof(double), hipMemcpyDeviceToHost, st));
            RBF_HIP(hipStreamSynchronize(st));
            double ss = 0.0;
            for (double v : hp) ss += v;
            const double nrm = std::sqrt(ss);
            if (!(nrm > 0.0) || !std::isfinite(nrm)) {
                nu = 0.0;
                break;
            }
            nu = nrm;  // ||W A_s x|| with ||x|| = 1 from the second step on
            scale = 1.0 / nrm;
            std::swap(P.x, P.y);
        }
        const double nus = 1.05 * nu;
        double w2 = (nus > 1.0) ? 0.85 / (nus - 1.0) : 1.6;
        S->ax64.w2 = (nu > 0.0) ? std::min(1.6, std::max(1.0, w2)) : 1.0;
    }
    if (S->mixed) {
        float *w32, *dinv32, *sinv32, *rval32;
        const int64_t nw = (int64_t)S->k * M;
        ALLOC(w32, nw);
        ALLOC(dinv32, M);
        ALLOC(sinv32, M);
        ALLOC(rval32, std::max<size_t>(1, rval.size()));
        const dim3 gc(1024), bc(256);
        hipLaunchKernelGGL(k_aux_to_f32, gc, bc, 0, st, nw, S->p_w, w32);
        hipLaunchKernelGGL(k_aux_to_f32, gc, bc, 0, st, M, ddinv, dinv32);
        hipLaunchKernelGGL(k_aux_to_f32, gc, bc, 0, st, M, dsinv, sinv32);
        if (!rval.empty())
            hipLaunchKernelGGL(k_aux_to_f32, gc, bc, 0, st, (int64_t)rval.size(), drval, rval32);
        RBF_CHECK_LAUNCH();
        S->p_w32 = w32;
        S->ax32 = AuxOps<float>{S->idx_pp, w32, dinv32, sinv32, drptr, drcol, rval32, M, S->k};
        S->ax32.w2 = S->ax64.w2;
        if ((rc = alloc_fg(S, S->fg32, M)) != RBF_OK) return rc;
        L.flag = S->fg32.s.flag;
    } else {
        if ((rc = alloc_fg(S, S->fg64, M)) != RBF_OK) return rc;
        L.flag = S->fg64.s.flag;
    }
    RBF_HIP(hipStreamSynchronize(st));
    S->aux_K = Ka;
    S->aux_on = true;
    return RBF_OK;
}

// ------------------------------------------------------- diagnostics --
// Maximum that propagates NaN (a non-finite field must show in the result).
__device__ __forceinline__ double nanmax(double a, double b) {
    return (a != a || b != b) ? __builtin_nan("") : fmax(a, b);
}
__device__ __forceinline__ double block_max(double v) {
    __shared__ double lds[kThreads / 64];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = nanmax(v, __shfl_xor(v, off, 64));
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
    __syncthreads();
    double m = lds[0];
    for (int w = 1; w < kThreads / 64; ++w) m = nanmax(m, lds[w]);
    __syncthreads();
    return m;
}

// Distance from each V-node to its nearest stencil neighbour (CFL scale).
__global__ void __launch_bounds__(kThreads) k_vhmin(int64_t n, int k, const int *__restrict__ idx,
                                                     const double *__restrict__ xv,
                                                     double *__restrict__ hmin) {
    const int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (r >= n) return;
    const double x = xv[r], y = xv[n + r];
    double d2 = __builtin_inf();
    for (int s = 0; s < k; ++s) {
        const int j = idx[(int64_t)s * n + r];
        if (j == r) continue;
        const double dx = xv[j] - x, dy = xv[n + j] - y;
        d2 = fmin(d2, dx * dx + dy * dy);
    }
    hmin[r] = sqrt(d2);
}

// V rows: block partials of sum(u^2 + v^2), max speed, max speed / hmin.
__global__ void __launch_bounds__(kThreads) k_diag_v(int64_t n, const double *__restrict__ u,
                                                      const double *__restrict__ v,
                                                      const double *__restrict__ hmin,
                                                      double *__restrict__ part) {
    double s[1] = {0.0}, smax = 0.0, cmax = 0.0;
    for (int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * kThreads) {
        const double q = u[r] * u[r] + v[r] * v[r], sp = sqrt(q);
        s[0] += q;
        smax = nanmax(smax, sp);
        cmax = nanmax(cmax, sp / hmin[r]);
    }
    smax = block_max(smax);
    cmax = block_max(cmax);
    {
        __shared__ double lds[kThreads / 64];
        rbf::block_sum<1>(s, lds);
    }
    if (threadIdx.x == 0) {
        part[blockIdx.x] = s[0];
        part[gridDim.x + blockIdx.x] = smax;
        part[2 * gridDim.x + blockIdx.x] = cmax;
    }
}

// Interior P rows: F = D_x^PV u + D_y^PV v (eq. (17)); block partials of
// max |F| and sum F^2.
template <int KT>
__global__ void __launch_bounds__(kThreads) k_diag_p(int64_t m, int k, const int *__restrict__ idx,
                                                      const double *__restrict__ wdx,
                                                      const double *__restrict__ wdy,
                                                      const double *__restrict__ u,
                                                      const double *__restrict__ v,
                                                      const int8_t *__restrict__ ptag,
                                                      double *__restrict__ part) {
    double s2[1] = {0.0}, fmx = 0.0;
    const double *ws[2] = {wdx, wdy};
    for (int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x; r < m;
         r += (int64_t)gridDim.x * kThreads) {
        if (ptag[r] != 0) continue;
        double acc[2][2] = {};
        rbf::ell_row<KT, 2>(idx, ws, m, r, k, Gather2{u, v}, acc);
        const double F = acc[0][0] + acc[1][1];
        fmx = nanmax(fmx, fabs(F));
        s2[0] += F * F;
    }
    fmx = block_max(fmx);
    {
        __shared__ double lds[kThreads / 64];
        rbf::block_sum<1>(s2, lds);
    }
    if (threadIdx.x == 0) {
        part[blockIdx.x] = fmx;
        part[gridDim.x + blockIdx.x] = s2[0];
    }
}

// Lowest ELL position of idx[0, n) outside [0, ns) into *bad (atomic min).
__global__ void k_idx_range(const int *__restrict__ idx, int64_t n, int64_t ns,
                            unsigned long long *bad) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int c = idx[e];
        if (c < 0 || (int64_t)c >= ns) atomicMin(bad, (unsigned long long)e);
    }
}

// Every stencil index of the four operators lies in its source node range;
// checked before any kernel gathers through them.
rbf_status check_stencils(hipStream_t st, const rbf_grid *g, const rbf_ops *o) {
    struct Set {
        const char *name;
        const int *idx;
        int64_t rows, ns;
    };
    const Set sets[4] = {{"idx_vv", o->idx_vv, g->n_v, g->n_v},
                         {"idx_pv", o->idx_pv, g->n_p, g->n_v},
                         {"idx_pp", o->idx_pp, g->n_p, g->n_p},
                         {"idx_vp", o->idx_vp, g->n_v, g->n_p}};
    unsigned long long *bad = nullptr;
    RBF_HIP(hipMalloc((void **)&bad, 4 * sizeof(unsigned long long)));
    unsigned long long hb[4];
    int hv[4] = {0, 0, 0, 0};
    rbf_status rc = RBF_OK;
    auto run = [&]() -> rbf_status {
        RBF_HIP(hipMemsetAsync(bad, 0xff, 4 * sizeof(unsigned long long), st));
        for (int q = 0; q < 4; ++q) {
            const int64_t n = sets[q].rows * o->k;
            hipLaunchKernelGGL(k_idx_range, dim3(std::min<uint32_t>(rbf::blocks_for(n, 256), 4096u)),
                               dim3(256), 0, st, sets[q].idx, n, sets[q].ns, bad + q);
        }
        RBF_CHECK_LAUNCH();
        RBF_HIP(hipMemcpyAsync(hb, bad, sizeof(hb), hipMemcpyDeviceToHost, st));
        RBF_HIP(hipStreamSynchronize(st));
        for (int q = 0; q < 4; ++q)
            if (hb[q] != ~0ull) {
                RBF_HIP(hipMemcpy(&hv[q], sets[q].idx + hb[q], sizeof(int), hipMemcpyDeviceToHost));
                rbf::set_error("rbf_solver_create: %s[%llu][%llu] = %d is outside [0, %lld)",
                               sets[q].name, hb[q] / (unsigned long long)sets[q].rows,
                               hb[q] % (unsigned long long)sets[q].rows, hv[q],
                               (long long)sets[q].ns);
                return RBF_E_ARG;
            }
        return RBF_OK;
    };
    rc = run();
    if (rc != RBF_OK) (void)hipStreamSynchronize(st);
    (void)hipFree(bad);
    return rc;
}

rbf_status create_impl(rbf_solver *S, const rbf_grid *g, const rbf_ops *o, const double *u_bc,
                       const double *v_bc, const rbf_params *prm) {
    const int64_t N = g->n_v, M = g->n_p;
    const int k = o->k;
    S->N = N;
    S->M = M;
    S->k = k;
    S->re = prm->re;
    S->dt = prm->dt;
    S->a = prm->dt / (2.0 * prm->re);
    S->rtol_h = prm->rtol_h;
    S->rtol_p = prm->rtol_p;
    S->maxit_h = prm->maxit_h;
    S->maxit_p = prm->maxit_p;
    S->mixed = (prm->precision == RBF_PRECISION_MIXED);
    const int64_t kN = (int64_t)k * N, kM = (int64_t)k * M;
    ALLOC(S->idx_vv, kN);
    ALLOC(S->idx_pv, kM);
    ALLOC(S->idx_pp, kM);
    ALLOC(S->idx_vp, kN);
    ALLOC(S->vv_dx, kN);
    ALLOC(S->vv_dy, kN);
    ALLOC(S->vv_lap, kN);
    ALLOC(S->pv_dx, kM);
    ALLOC(S->pv_dy, kM);
    ALLOC(S->pp_lap, kM);
    ALLOC(S->vp_dx, kN);
    ALLOC(S->vp_dy, kN);
    ALLOC(S->h_w, kN);
    ALLOC(S->h_dinv, N);
    ALLOC(S->p_w, kM);
    ALLOC(S->p_dinv, M);
    ALLOC(S->p_rowscale, M);
    ALLOC(S->p_u1, M);
    ALLOC(S->p_warm, M);
    ALLOC(S->p_prev, M);
    ALLOC(S->p_prev2, M);
    ALLOC(S->p_prev3, M);
    for (double *&q : S->hh) ALLOC(q, 2 * N);
    ALLOC(S->p_rhs_tmp, M);
    ALLOC(S->p_tag, M);
    ALLOC(S->u_bc, N);
    ALLOC(S->v_bc, N);
    ALLOC(S->wall_rows, N);
    ALLOC(S->v_hmin, N);
    ALLOC(S->diag_part, 5 * kMaxBlocks);
    for (double **q : {&S->u, &S->v, &S->cu, &S->cv, &S->un, &S->vn, &S->cun, &S->cvn, &S->us, &S->vs})
        ALLOC(*q, N);
    for (double **q : {&S->pt, &S->p, &S->ptn, &S->pn, &S->prhs}) ALLOC(*q, M);
    ALLOC(S->hrhs, 2 * N);
    ALLOC(S->uvss, 2 * N);
    ALLOC(S->rpart, kMaxNR * kMaxBlocks);
    rbf_status rc;
    {
        HKry &H = S->hk;
        for (double **q : {&H.r, &H.rh, &H.p[0], &H.p[1], &H.v, &H.s, &H.t, &H.ph, &H.sh})
            ALLOC(*q, kHR * N);
        ALLOC(H.partI, 2 * kHR * kMaxBlocks);
        ALLOC(H.part1, kHR * kMaxBlocks);
        ALLOC(H.part3, kHR * kMaxBlocks);
        ALLOC(H.part6, 3 * kHR * kMaxBlocks);
        ALLOC(H.rec, (int64_t)(S->maxit_h + 2) * kHR * 4);
        ALLOC(H.bb, kHR);
        ALLOC(H.rhrh, kHR);
        ALLOC(H.best, 2 * kHR * 2);
        ALLOC(H.flag, kHR);
        JKry &J = S->jk;
        ALLOC(J.x[0], kHR * N);
        ALLOC(J.x[1], kHR * N);
        ALLOC(J.part, 2 * 2 * kHR * kMaxBlocks);
        ALLOC(J.bb, kHR);
        ALLOC(J.flag, 2);
        ALLOC(H.iters, kHR);
    }
    if ((rc = alloc_krylov(S, S->kp, 1, M, S->maxit_p)) != RBF_OK) return rc;
    RBF_HIP(hipHostMalloc((void **)&S->hflag, 64 * sizeof(int), hipHostMallocDefault));
    RBF_HIP(hipHostMalloc((void **)&S->hred, (2 * kMaxNR * kMaxBlocks + kMaxNR) * sizeof(double),
                          hipHostMallocDefault));

    const size_t ib = sizeof(int), db = sizeof(double);
    struct {
        void *d;
        const void *s;
        size_t b;
    } cp[] = {{S->idx_vv, o->idx_vv, kN * ib}, {S->idx_pv, o->idx_pv, kM * ib},
              {S->idx_pp, o->idx_pp, kM * ib}, {S->idx_vp, o->idx_vp, kN * ib},
              {S->vv_dx, o->vv_dx, kN * db},   {S->vv_dy, o->vv_dy, kN * db},
              {S->vv_lap, o->vv_lap, kN * db}, {S->pv_dx, o->pv_dx, kM * db},
              {S->pv_dy, o->pv_dy, kM * db},   {S->pp_lap, o->pp_lap, kM * db},
              {S->vp_dx, o->vp_dx, kN * db},   {S->vp_dy, o->vp_dy, kN * db},
              {S->p_tag, g->p_tag, (size_t)M}, {S->u_bc, u_bc, N * db},
              {S->v_bc, v_bc, N * db}};
    for (auto &c : cp)
        if ((rc = copy_in(S, c.d, c.s, c.b)) != RBF_OK) return rc;

    hipStream_t st = S->st;
    int *err, *cnt;
    ALLOC(err, 1);
    ALLOC(cnt, 1);
    RBF_HIP(hipMemsetAsync(err, 0, sizeof(int), st));
    RBF_HIP(hipMemsetAsync(cnt, 0, sizeof(int), st));
    hipLaunchKernelGGL(k_build_helmholtz, dim3(rbf::blocks_for(N, 256)), dim3(256), 0, st, N, k,
                       S->idx_vv, S->vv_lap, g->v_tag, S->a, S->h_w, S->h_dinv, err);
    hipLaunchKernelGGL(k_build_poisson, dim3(rbf::blocks_for(M, 256)), dim3(256), 0, st, M, k,
                       S->idx_pp, S->pp_lap, o->pp_dx, o->pp_dy, g->p_tag, g->p_normal,
                       S->p_w, S->p_dinv, S->p_rowscale, S->p_u1, err);
    hipLaunchKernelGGL(k_wall_list, dim3(rbf::blocks_for(N, 256)), dim3(256), 0, st, N, g->v_tag,
                       S->wall_rows, cnt);
    hipLaunchKernelGGL(k_vhmin, dim3(rbf::blocks_for(N, kThreads)), dim3(kThreads), 0, st, N, k,
                       S->idx_vv, g->xv, S->v_hmin);
    RBF_CHECK_LAUNCH();
    int herr[2] = {0, 0};
    RBF_HIP(hipMemcpyAsync(&herr[0], err, ib, hipMemcpyDeviceToHost, st));
    RBF_HIP(hipMemcpyAsync(&herr[1], cnt, ib, hipMemcpyDeviceToHost, st));
    RBF_HIP(hipStreamSynchronize(st));
    RBF_ARG(herr[0] == 0, "rbf_solver_create: a %s stencil does not contain its own node (or a zero row)",
            (herr[0] & 1) ? "(V,V)" : "(P,P)");
    S->nwall = herr[1];
    {  // open boundary rows (outflow, symmetry): keep the tags on the device
        std::vector<int8_t> vt(N);
        RBF_HIP(hipMemcpyAsync(vt.data(), g->v_tag, N, hipMemcpyDeviceToHost, st));
        RBF_HIP(hipStreamSynchronize(st));
        bool open = false;
        for (int64_t r = 0; r < N && !open; ++r)
            open = vt[r] == RBF_VTAG_OUTFLOW || vt[r] == RBF_VTAG_SYMMETRY;
        if (open) {
            RBF_ARG(std::isfinite(prm->u_conv), "rbf_solver_create: u_conv must be finite");
            ALLOC(S->v_tag_open, N);
            RBF_HIP(hipMemcpyAsync(S->v_tag_open, vt.data(), N, hipMemcpyHostToDevice, st));
            S->u_conv = prm->u_conv;
        }
    }
    {  // infinity norm of the Jacobi iteration matrix of H
        const int nbb = (int)rbf::blocks_for(N, 256);
        double *bpart;
        ALLOC(bpart, nbb);
        hipLaunchKernelGGL(k_jacobi_bound, dim3(nbb), dim3(256), 0, st, N, k, S->idx_vv, S->h_w,
                           S->h_dinv, bpart);
        RBF_CHECK_LAUNCH();
        std::vector<double> hb(nbb);
        RBF_HIP(hipMemcpyAsync(hb.data(), bpart, nbb * sizeof(double), hipMemcpyDeviceToHost, st));
        RBF_HIP(hipStreamSynchronize(st));
        double bound = 0.0;
        for (double v : hb) bound = std::isfinite(v) ? std::max(bound, v) : INFINITY;
        S->h_bound = bound;
        S->h_jacobi = bound <= kJacobiMax;
    }
    if (S->mixed && S->h_jacobi) {
        HMix &X = S->hm;
        float *w32 = nullptr, *d32 = nullptr;
        ALLOC(w32, (int64_t)k * N);
        ALLOC(d32, N);
        ALLOC(X.x, N);
        ALLOC(X.r, N);
        ALLOC(X.d[0], N);
        ALLOC(X.d[1], N);
        ALLOC(X.part, 2 * 2 * kHR * kMaxBlocks);
        ALLOC(X.flag, 2);
        const dim3 gc(rbf::blocks_for((int64_t)k * N, 256)), bc(256);
        hipLaunchKernelGGL(k_aux_to_f32, gc, bc, 0, st, (int64_t)k * N, S->h_w, w32);
        hipLaunchKernelGGL(k_aux_to_f32, dim3(rbf::blocks_for(N, 256)), bc, 0, st, N, S->h_dinv, d32);
        RBF_CHECK_LAUNCH();
        X.idx = S->idx_vv;
        X.w32 = w32;
        X.dinv32 = d32;
        X.n = N;
        X.k = k;
        S->h_mixed = true;
    }
    // Scale of the zero-mean border: v = gamma / M with gamma = 1 / mean |u1|
    // over interior rows, so the border couples at the scale of the rows.
    std::vector<double> hu(M);
    RBF_HIP(hipMemcpyAsync(hu.data(), S->p_u1, M * db, hipMemcpyDeviceToHost, st));
    RBF_HIP(hipStreamSynchronize(st));
    double su = 0.0;
    int64_t ni = 0;
    for (int64_t r = 0; r < M; ++r)
        if (hu[r] != 0.0) {
            su += std::fabs(hu[r]);
            ++ni;
        }
    RBF_ARG(ni > 0, "rbf_solver_create: no interior P-node");
    S->n_interior_p = ni;
    S->p_vscale = ((double)ni / su) / (double)M;
    // The wall list order from atomics is irrelevant: rows are independent.
    rc = setup_lattice_pc(S, g, prm->precond);
    if (rc != RBF_OK) return rc;
    return setup_aux_pc(S, g, prm->precond);
}

rbf_status step_once(rbf_solver *S, bool first, rbf_step_stats *stats) {
    hipStream_t st = S->st;
    const int64_t N = S->N, M = S->M;
    const int k = S->k;
    const dim3 gN(rbf::blocks_for(N, kThreads)), gM(rbf::blocks_for(M, kThreads)), blk(kThreads);
    // Stage 1.
    launch_kt(k, [&](auto KT) {
        hipLaunchKernelGGL((k_advect<decltype(KT)::value>), gN, blk, 0, st, N, k, S->idx_vv, S->vv_dx,
                           S->vv_dy, S->u, S->v, S->cu, S->cv, first ? 1 : 0, S->dt, S->us, S->vs,
                           S->cun, S->cvn);
        // Stage 2 right-hand side and initial guess.
        hipLaunchKernelGGL((k_helm_rhs<decltype(KT)::value>), gN, blk, 0, st, N, k, S->idx_vv, S->vv_lap, S->a,
                           S->us, S->vs, S->hrhs, S->uvss);
    });
    // Initial guess on interior rows: the previous solutions of this call,
    // extrapolated in time (wall rows get their values below).
    {
        const dim3 g2(rbf::blocks_for(2 * N, 256)), b2(256);
        if (S->have_h >= 4)
            hipLaunchKernelGGL(k_guess<4>, g2, b2, 0, st, 2 * N, S->uvss, S->hh[0], S->hh[1], S->hh[2], S->hh[3]);
        else if (S->have_h == 3)
            hipLaunchKernelGGL(k_guess<3>, g2, b2, 0, st, 2 * N, S->uvss, S->hh[0], S->hh[1], S->hh[2], S->hh[3]);
        else if (S->have_h == 2)
            hipLaunchKernelGGL(k_guess<2>, g2, b2, 0, st, 2 * N, S->uvss, S->hh[0], S->hh[1], S->hh[2], S->hh[3]);
        else if (S->have_h == 1)
            hipLaunchKernelGGL(k_guess<1>, g2, b2, 0, st, 2 * N, S->uvss, S->hh[0], S->hh[1], S->hh[2], S->hh[3]);
    }
    if (S->nwall > 0)
        launch_kt(k, [&](auto KT) {
            // Wall rows are few and scattered (uncoalesced gathers): small
            // workgroups spread them over more compute units.
            hipLaunchKernelGGL((k_wall_rhs<decltype(KT)::value>),
                               dim3(rbf::blocks_for(S->nwall, 64)), dim3(64), 0, st, S->nwall,
                               S->wall_rows, N, k, S->idx_vp, S->vp_dx, S->vp_dy, S->pt, S->u_bc,
                               S->v_bc, S->dt, S->hrhs, S->uvss,
                               OpenBc{S->v_tag_open, S->idx_vv, S->vv_dx, S->vv_dy, S->u, S->v,
                                      S->u_conv});
        });
    RBF_CHECK_LAUNCH();
    rbf_solve_stats hs[2];
    EllM H{S->idx_vv, S->h_w, S->h_dinv, N, k, nullptr, 0.0};
    rbf_status rc = S->h_mixed
                        ? hmixed(S, H, S->hrhs, S->uvss, S->rtol_h, S->maxit_h, S->last_iters_h, hs)
                    : S->h_jacobi
                        ? hjacobi(S, H, S->hrhs, S->uvss, S->rtol_h, S->maxit_h, S->last_iters_h, hs)
                        : hbicgstab(S, H, S->hrhs, S->uvss, S->rtol_h, S->maxit_h, S->last_iters_h, hs);
    if (stats) {
        stats->last_helmholtz_u = hs[0];
        stats->last_helmholtz_v = hs[1];
        stats->helmholtz_iters += hs[0].iterations + hs[1].iterations;
    }
    if (rc != RBF_OK) return rc;
    // Stage 3: divergence, Poisson (warm start from p~_j), pressure, correction.
    launch_kt(k, [&](auto KT) {
        hipLaunchKernelGGL((k_divergence<decltype(KT)::value>), gM, blk, 0, st, M, k, S->idx_pv, S->pv_dx,
                           S->pv_dy, S->uvss, S->uvss + N, S->p_tag, 1.0 / S->dt,
                           S->p_rowscale, S->prhs);
    });
    // Initial guess: the previous solutions of this call extrapolated in
    // time (up to cubic, from the last four).
    if (S->have_prev >= 3) {
        hipLaunchKernelGGL(k_extrapolate<3>, dim3(rbf::blocks_for(M, 256)), dim3(256), 0, st, M,
                           S->p_warm, S->p_prev, S->p_prev2, S->p_prev3);
    } else if (S->have_prev == 2) {
        hipLaunchKernelGGL(k_extrapolate<2>, dim3(rbf::blocks_for(M, 256)), dim3(256), 0, st, M,
                           S->p_warm, S->p_prev, S->p_prev2, S->p_prev3);
        S->have_prev = 3;
    } else if (S->have_prev == 1) {
        hipLaunchKernelGGL(k_extrapolate<1>, dim3(rbf::blocks_for(M, 256)), dim3(256), 0, st, M,
                           S->p_warm, S->p_prev, S->p_prev2, S->p_prev3);
        S->have_prev = 2;
    } else {
        RBF_HIP(hipMemcpyAsync(S->p_prev, S->p_warm, M * sizeof(double), hipMemcpyDeviceToDevice, st));
        S->have_prev = 1;
    }
    rbf_solve_stats ps;
    rc = poisson_solve(S, S->prhs, S->p_warm, &ps);
    if (rc == RBF_OK) {  // p~ = solution minus its mean (zero-mean border)
        const int nbm = nblocks_rows(M);
        hipLaunchKernelGGL((k_sum<1>), dim3(nbm), dim3(kThreads), 0, st, M, S->p_warm, S->kp.partX);
        hipLaunchKernelGGL(k_sub_mean, dim3(nbm), dim3(kThreads), 0, st, M, S->kp.partX, nbm,
                           S->p_warm, S->ptn);
    }
    if (stats) {
        stats->last_poisson = ps;
        stats->poisson_iters += ps.iterations;
    }
    if (rc != RBF_OK) return rc;
    launch_kt(k, [&](auto KT) {
        hipLaunchKernelGGL((k_pressure<decltype(KT)::value>), gM, blk, 0, st, M, k, S->idx_pp, S->pp_lap, S->a,
                           S->ptn, S->pn);
        hipLaunchKernelGGL((k_correct<decltype(KT)::value>), gN, blk, 0, st, N, k, S->idx_vp, S->vp_dx,
                           S->vp_dy, S->dt, S->ptn, S->uvss, S->un, S->vn);
    });
    RBF_CHECK_LAUNCH();
    // Commit.  The viscous solution joins the history of initial guesses by
    // pointer rotation; the oldest history buffer becomes the next step's
    // workspace.
    {
        double *oldest = S->hh[3];
        S->hh[3] = S->hh[2];
        S->hh[2] = S->hh[1];
        S->hh[1] = S->hh[0];
        S->hh[0] = S->uvss;
        S->uvss = oldest;
        S->have_h = std::min(S->have_h + 1, 4);
    }
    std::swap(S->u, S->un);
    std::swap(S->v, S->vn);
    std::swap(S->pt, S->ptn);
    std::swap(S->p, S->pn);
    std::swap(S->cu, S->cun);
    std::swap(S->cv, S->cvn);
    return RBF_OK;
}

}  // namespace

extern "C" rbf_status rbf_solver_create(rbf_solver **out, const rbf_grid *grid, const rbf_ops *ops,
                                        const double *u_bc, const double *v_bc,
                                        const rbf_params *prm, rbf_stream st) {
    rbf::clear_error();
    RBF_ARG(out && grid && ops && prm && u_bc && v_bc, "rbf_solver_create: NULL argument");
    *out = nullptr;
    RBF_ARG(grid->n_v > 0 && grid->n_p > 0 && grid->n_v < INT32_MAX && grid->n_p < INT32_MAX,
            "rbf_solver_create: node counts out of range");
    RBF_ARG(grid->xv && grid->xp && grid->v_tag && grid->p_tag && grid->p_normal,
            "rbf_solver_create: NULL grid array");
    RBF_ARG(ops->k >= 1 && ops->k <= 64 && ops->k <= grid->n_v && ops->k <= grid->n_p,
            "rbf_solver_create: stencil size out of range");
    RBF_ARG(ops->idx_vv && ops->vv_dx && ops->vv_dy && ops->vv_lap && ops->idx_pv && ops->pv_dx &&
                ops->pv_dy && ops->idx_pp && ops->pp_dx && ops->pp_dy && ops->pp_lap &&
                ops->idx_vp && ops->vp_dx && ops->vp_dy,
            "rbf_solver_create: NULL operator array");
    RBF_ARG(prm->re > 0 && prm->dt > 0 && std::isfinite(prm->re) && std::isfinite(prm->dt),
            "rbf_solver_create: re and dt must be positive");
    RBF_ARG(prm->rtol_h > 0 && prm->rtol_p > 0, "rbf_solver_create: tolerances must be positive");
    RBF_ARG(prm->maxit_h >= 1 && prm->maxit_p >= 1 && prm->maxit_h <= 1000000 &&
                prm->maxit_p <= 1000000,
            "rbf_solver_create: iteration caps out of range");
    RBF_ARG(prm->precision == RBF_PRECISION_FP64 || prm->precision == RBF_PRECISION_MIXED,
            "rbf_solver_create: unknown precision %d", prm->precision);
    RBF_ARG(prm->precond == RBF_PRECOND_AUTO || prm->precond == RBF_PRECOND_NONE ||
                prm->precond == RBF_PRECOND_LATTICE || prm->precond == RBF_PRECOND_AUX,
            "rbf_solver_create: unknown precond %d", prm->precond);
    rbf_solver *S = new rbf_solver();
    S->st = rbf::as_stream(st);
    if (hipGetDevice(&S->device) != hipSuccess) {
        delete S;
        rbf::set_error("rbf_solver_create: hipGetDevice failed");
        return RBF_E_DEVICE;
    }
    rbf_status rc = check_stencils(S->st, grid, ops);
    if (rc == RBF_OK) rc = create_impl(S, grid, ops, u_bc, v_bc, prm);
    if (rc != RBF_OK) {
        rbf_solver_destroy(S);
        return rc;
    }
    *out = S;
    return RBF_OK;
}

extern "C" rbf_status rbf_step(rbf_solver *S, int32_t nsteps, rbf_state *state,
                               rbf_step_stats *stats) {
    rbf::clear_error();
    RBF_ARG(S && state, "rbf_step: NULL argument");
    RBF_ARG(nsteps >= 0, "rbf_step: nsteps < 0");
    RBF_ARG(state->u && state->v && state->p_tilde && state->p && state->cu_prev && state->cv_prev,
            "rbf_step: NULL state array");
    if (stats) *stats = rbf_step_stats{};
    const size_t nb = S->N * sizeof(double), mb = S->M * sizeof(double);
    hipStream_t st = S->st;
    RBF_HIP(hipMemcpyAsync(S->u, state->u, nb, hipMemcpyDeviceToDevice, st));
    RBF_HIP(hipMemcpyAsync(S->v, state->v, nb, hipMemcpyDeviceToDevice, st));
    RBF_HIP(hipMemcpyAsync(S->cu, state->cu_prev, nb, hipMemcpyDeviceToDevice, st));
    RBF_HIP(hipMemcpyAsync(S->cv, state->cv_prev, nb, hipMemcpyDeviceToDevice, st));
    RBF_HIP(hipMemcpyAsync(S->pt, state->p_tilde, mb, hipMemcpyDeviceToDevice, st));
    RBF_HIP(hipMemcpyAsync(S->p_warm, state->p_tilde, mb, hipMemcpyDeviceToDevice, st));
    S->have_prev = 0;
    S->have_h = 0;
    RBF_HIP(hipMemcpyAsync(S->p, state->p, mb, hipMemcpyDeviceToDevice, st));
    rbf_status rc = RBF_OK;
    int done = 0;
    for (; done < nsteps; ++done) {
        rc = step_once(S, state->step + done == 0, stats);
        if (stats) stats->status = rc;
        if (rc != RBF_OK) break;
    }
    if (stats) stats->steps_done = done;
    if (done > 0) {
        RBF_HIP(hipMemcpyAsync(state->u, S->u, nb, hipMemcpyDeviceToDevice, st));
        RBF_HIP(hipMemcpyAsync(state->v, S->v, nb, hipMemcpyDeviceToDevice, st));
        RBF_HIP(hipMemcpyAsync(state->cu_prev, S->cu, nb, hipMemcpyDeviceToDevice, st));
        RBF_HIP(hipMemcpyAsync(state->cv_prev, S->cv, nb, hipMemcpyDeviceToDevice, st));
        RBF_HIP(hipMemcpyAsync(state->p_tilde, S->pt, mb, hipMemcpyDeviceToDevice, st));
        RBF_HIP(hipMemcpyAsync(state->p, S->p, mb, hipMemcpyDeviceToDevice, st));
        state->step += done;
    }
    RBF_HIP(hipStreamSynchronize(st));
    return rc;
}

// ------------------------------------------------------- adjoint step --
namespace {

// Column structure and column-ordered weights of the transposes (once).
rbf_status adj_transpose(rbf_solver *S, int64_t rows, const int *idx, int64_t ncols,
                         std::initializer_list<std::pair<const double *, double **>> ws,
                         int64_t **cp, int **src) {
    const int k = S->k;
    int *slot;
    ALLOC(*cp, ncols + 1);
    ALLOC(*src, (int64_t)k * rows);
    ALLOC(slot, (int64_t)k * rows);
    int64_t bad = -1;
    rbf_status rc = rbf_ell_transpose(rows, k, idx, ncols, *cp, *src, slot, &bad, S->st);
    if (rc != RBF_OK) return rc;
    for (auto &pw : ws) {
        ALLOC(*pw.second, (int64_t)k * rows);
        if ((rc = rbf_ell_transpose_weights(rows, k, *src, slot, pw.first, *pw.second, 0, S->st)) !=
            RBF_OK)
            return rc;
    }
    return RBF_OK;
}

rbf_status adj_setup(rbf_solver *S) {
    auto &A = S->adj;
    const int64_t N = S->N, M = S->M;
    rbf_status rc;
    if ((rc = adj_transpose(S, N, S->idx_vv, N,
                            {{S->vv_dx, &A.dxT_vv}, {S->vv_dy, &A.dyT_vv}, {S->vv_lap, &A.lapT_vv}},
                            &A.cp_vv, &A.src_vv)) != RBF_OK)
        return rc;
    if ((rc = adj_transpose(S, N, S->idx_vp, M, {{S->vp_dx, &A.dxT_vp}, {S->vp_dy, &A.dyT_vp}},
                            &A.cp_vp, &A.src_vp)) != RBF_OK)
        return rc;
    if ((rc = adj_transpose(S, M, S->idx_pv, N, {{S->pv_dx, &A.dxT_pv}, {S->pv_dy, &A.dyT_pv}},
                            &A.cp_pv, &A.src_pv)) != RBF_OK)
        return rc;
    if ((rc = adj_transpose(S, M, S->idx_pp, M, {{S->p_w, &A.aT_pp}}, &A.cp_pp, &A.src_pp)) !=
        RBF_OK)
        return rc;
    ALLOC(A.vtag, N);
    RBF_HIP(hipMemsetAsync(A.vtag, 0, N, S->st));
    if (S->nwall > 0)
        hipLaunchKernelGGL(k_adj_wallmask, dim3(rbf::blocks_for(S->nwall, 256)), dim3(256), 0,
                           S->st, S->nwall, S->wall_rows, A.vtag);
    for (auto &q : A.vn) ALLOC(q, N);
    for (auto &q : A.pm) ALLOC(q, M);
    for (auto &q : A.kr) ALLOC(q, std::max(N, M));
    ALLOC(A.part, 4 * kMaxBlocks);
    RBF_HIP(hipStreamSynchronize(S->st));
    A.ready = true;
    return RBF_OK;
}

// NQ dot products (or sums) over n entries, reduced on the host in a fixed
// order (synchronises).
template <int NQ>
rbf_status adj_dots(rbf_solver *S, int64_t n, AdjDots d, double *out) {
    const int nb = nblocks_rows(n);
    hipLaunchKernelGGL(k_adj_dots<NQ>, dim3(nb), dim3(kThreads), 0, S->st, n, d, S->adj.part);
    RBF_CHECK_LAUNCH();
    for (int q = 0; q < NQ; ++q)
        RBF_HIP(hipMemcpyAsync(S->hred + q * nb, S->adj.part + (int64_t)q * kMaxBlocks,
                               nb * sizeof(double), hipMemcpyDeviceToHost, S->st));
    RBF_HIP(hipStreamSynchronize(S->st));
    for (int q = 0; q < NQ; ++q) {
        double acc = 0.0;
        for (int b = 0; b < nb; ++b) acc += S->hred[q * nb + b];
        out[q] = acc;
    }
    return RBF_OK;
}

void adj_axpby(rbf_solver *S, int64_t n, double a, const double *x, double b, const double *y,
               double *out) {
    hipLaunchKernelGGL(k_adj_axpby, dim3(std::min<int64_t>(1024, rbf::blocks_for(n, 256))),
                       dim3(256), 0, S->st, n, a, x, b, y, out);
}

// BiCGSTAB (van der Vorst 1992) for op(x) = b from x = 0, with the
// Jacobi-type diagonal scaling dinv (nullable) as right preconditioner.
// Scalars are reduced on the host (a few synchronisations per iteration):
// these solves run once per adjoint step.
template <class Op>
rbf_status adj_bicgstab(rbf_solver *S, int64_t n, Op op, const double *dinv, const double *b,
                        double *x, double tol, int maxit, const char *what) {
    auto &K = S->adj.kr;
    double *r = K[0], *rh = K[1], *p = K[2], *v = K[3], *s = K[4], *t = K[5], *z = K[6];
    auto prec = [&](const double *in, double *out) {
        if (dinv) hipLaunchKernelGGL(k_adj_mul, dim3(std::min<int64_t>(1024, rbf::blocks_for(n, 256))),
                                     dim3(256), 0, S->st, n, dinv, in, out);
        else RBF_HIP(hipMemcpyAsync(out, in, n * sizeof(double), hipMemcpyDeviceToDevice, S->st));
        return RBF_OK;
    };
    rbf_status rc;
    RBF_HIP(hipMemsetAsync(x, 0, n * sizeof(double), S->st));
    RBF_HIP(hipMemcpyAsync(r, b, n * sizeof(double), hipMemcpyDeviceToDevice, S->st));
    RBF_HIP(hipMemcpyAsync(rh, b, n * sizeof(double), hipMemcpyDeviceToDevice, S->st));
    RBF_HIP(hipMemsetAsync(p, 0, n * sizeof(double), S->st));
    RBF_HIP(hipMemsetAsync(v, 0, n * sizeof(double), S->st));
    double bb;
    if ((rc = adj_dots<1>(S, n, AdjDots{{b}, {b}}, &bb)) != RBF_OK) return rc;
    if (bb == 0.0) return RBF_OK;
    double rho = 1.0, alpha = 1.0, omega = 1.0;
    for (int it = 0; it < maxit; ++it) {
        double q[2];
        if ((rc = adj_dots<2>(S, n, AdjDots{{rh, r}, {r, r}}, q)) != RBF_OK) return rc;
        if (!std::isfinite(q[1])) {
            rbf::set_error("%s: non-finite residual (iteration %d)", what, it);
            return RBF_E_NAN;
        }
        if (q[1] <= tol * tol * bb) return RBF_OK;
        const double rho1 = q[0];
        if (it > 0 && std::fabs(rho1) < 1e-300) break;
        const double beta = (it == 0) ? 0.0 : (rho1 / rho) * (alpha / omega);
        rho = rho1;
        adj_axpby(S, n, 1.0, p, -omega, v, p);    // p - omega v
        adj_axpby(S, n, 1.0, r, beta, p, p);      // r + beta (p - omega v)
        if ((rc = prec(p, z)) != RBF_OK) return rc;
        if ((rc = op(z, v)) != RBF_OK) return rc;
        double rv;
        if ((rc = adj_dots<1>(S, n, AdjDots{{rh}, {v}}, &rv)) != RBF_OK) return rc;
        alpha = rho / rv;
        adj_axpby(S, n, 1.0, r, -alpha, v, s);
        adj_axpby(S, n, alpha, z, 1.0, x, x);     // x += alpha P p
        if ((rc = prec(s, z)) != RBF_OK) return rc;
        if ((rc = op(z, t)) != RBF_OK) return rc;
        double ts[2];
        if ((rc = adj_dots<2>(S, n, AdjDots{{t, t}, {s, t}}, ts)) != RBF_OK) return rc;
        omega = (ts[1] != 0.0) ? ts[0] / ts[1] : 0.0;
        adj_axpby(S, n, omega, z, 1.0, x, x);     // x += omega P s
        adj_axpby(S, n, 1.0, s, -omega, t, r);
        if (omega == 0.0) break;
    }
    // Final check of the true residual.
    if ((rc = op(x, t)) != RBF_OK) return rc;
    adj_axpby(S, n, 1.0, b, -1.0, t, t);
    double rr;
    if ((rc = adj_dots<1>(S, n, AdjDots{{t}, {t}}, &rr)) != RBF_OK) return rc;
    if (rr <= 100.0 * tol * tol * bb) return RBF_OK;
    rbf::set_error("%s: no convergence (relative residual %.3e after %d iterations)", what,
                   std::sqrt(rr / bb), maxit);
    return RBF_E_NOCONV;
}

}  // namespace

extern "C" rbf_status rbf_adjoint_step(rbf_solver *S, const rbf_state *fwd, rbf_state *adj,
                                       double *grad_bc, double *dnu) {
    rbf::clear_error();
    RBF_ARG(S && fwd && adj && grad_bc && dnu, "rbf_adjoint_step: NULL argument");
    RBF_ARG(!S->v_tag_open, "rbf_adjoint_step: needs Dirichlet boundary rows only (no outflow or symmetry rows)");
    RBF_ARG(fwd->u && fwd->v && fwd->p_tilde && fwd->cu_prev && fwd->cv_prev,
            "rbf_adjoint_step: NULL forward state array");
    RBF_ARG(adj->u && adj->v && adj->p_tilde && adj->cu_prev && adj->cv_prev,
            "rbf_adjoint_step: NULL adjoint state array");
    rbf_status rc;
    if (!S->adj.ready && (rc = adj_setup(S)) != RBF_OK) return rc;
    auto &A = S->adj;
    hipStream_t st = S->st;
    const int64_t N = S->N, M = S->M;
    const int k = S->k;
    const double dt = S->dt, a = S->a;
    const size_t nb = N * sizeof(double), mb = M * sizeof(double);
    const bool first = fwd->step == 0;
    // Forward step j -> j+1 again, from the caller's state, keeping u*, v*
    // (S->us, S->vs) and u**, v** (S->hh[0] after the commit).
    RBF_HIP(hipMemcpyAsync(S->u, fwd->u, nb, hipMemcpyDeviceToDevice, st));
    RBF_HIP(hipMemcpyAsync(S->v, fwd->v, nb, hipMemcpyDeviceToDevice, st));
    RBF_HIP(hipMemcpyAsync(S->cu, fwd->cu_prev, nb, hipMemcpyDeviceToDevice, st));
    RBF_HIP(hipMemcpyAsync(S->cv, fwd->cv_prev, nb, hipMemcpyDeviceToDevice, st));
    RBF_HIP(hipMemcpyAsync(S->pt, fwd->p_tilde, mb, hipMemcpyDeviceToDevice, st));
    RBF_HIP(hipMemcpyAsync(S->p_warm, fwd->p_tilde, mb, hipMemcpyDeviceToDevice, st));
    S->have_prev = 0;
    S->have_h = 0;
    if ((rc = step_once(S, first, nullptr)) != RBF_OK) return rc;
    const double *us = S->us, *vs = S->vs, *uss = S->hh[0], *vss = S->hh[0] + N;
    double **V = A.vn, **P = A.pm;
    double *ub = V[0], *vb = V[1], *rub = V[2], *rvb = V[3], *ri = V[4], *rw = V[5], *si = V[6],
           *sw = V[7], *t1 = V[8], *t2 = V[9], *usb = V[10], *vsb = V[11], *cub = V[12],
           *cvb = V[13], *qx = V[14], *qy = V[15], *px = V[16], *py = V[17], *t3 = V[18],
           *t4 = V[19];
    double *ptb = P[0], *y = P[1], *w = P[2], *fb = P[3], *m1 = P[4], *m2 = P[5];
    RBF_HIP(hipMemcpyAsync(ub, adj->u, nb, hipMemcpyDeviceToDevice, st));
    RBF_HIP(hipMemcpyAsync(vb, adj->v, nb, hipMemcpyDeviceToDevice, st));
    RBF_HIP(hipMemcpyAsync(ptb, adj->p_tilde, mb, hipMemcpyDeviceToDevice, st));
    RBF_HIP(hipMemcpyAsync(cub, adj->cu_prev, nb, hipMemcpyDeviceToDevice, st));
    RBF_HIP(hipMemcpyAsync(cvb, adj->cv_prev, nb, hipMemcpyDeviceToDevice, st));
    auto tvp = [&](const double *wt, const double *in, double *out) {  // out = D^VP^T in (M)
        return rbf_ell_apply_transpose(M, A.cp_vp, A.src_vp, wt, in, out, 0, st);
    };
    auto tpv = [&](const double *wt, const double *in, double *out) {  // out = D^PV^T in (N)
        return rbf_ell_apply_transpose(N, A.cp_pv, A.src_pv, wt, in, out, 0, st);
    };
    auto tvv = [&](const double *wt, const double *in, double *out) {  // out = D^VV^T in (N)
        return rbf_ell_apply_transpose(N, A.cp_vv, A.src_vv, wt, in, out, 0, st);
    };
    auto fvv = [&](const double *wv, const double *in, double *out) {  // out = D^VV in
        return rbf_ell_apply(N, k, S->idx_vv, wv, in, out, 0, st);
    };
#define ADJ(call)                           \
    do {                                    \
        if ((rc = (call)) != RBF_OK) return rc; \
    } while (0)
    // (20): p~_bar -= dt (Gx^T u_bar + Gy^T v_bar)
    ADJ(tvp(A.dxT_vp, ub, m1));
    ADJ(tvp(A.dyT_vp, vb, m2));
    adj_axpby(S, M, -dt, m1, 1.0, ptb, ptb);
    adj_axpby(S, M, -dt, m2, 1.0, ptb, ptb);
    // (18): (A_s + u1 c 1^T)^T w = p~_bar - mean(p~_bar); rhs_bar = S w
    double sm;
    ADJ(adj_dots<1>(S, M, AdjDots{{ptb}, {nullptr}}, &sm));
    hipLaunchKernelGGL(k_adj_addc, dim3(std::min<int64_t>(1024, rbf::blocks_for(M, 256))), dim3(256),
                       0, st, M, -sm / (double)M, ptb);
    RBF_HIP(hipMemcpyAsync(y, ptb, mb, hipMemcpyDeviceToDevice, st));
    const double c = S->p_vscale;
    auto pois_t = [&](const double *in, double *out) -> rbf_status {
        double d;
        rbf_status r2 = adj_dots<1>(S, M, AdjDots{{S->p_u1}, {in}}, &d);
        if (r2 != RBF_OK) return r2;
        r2 = rbf_ell_apply_transpose(M, A.cp_pp, A.src_pp, A.aT_pp, in, out, 0, st);
        if (r2 != RBF_OK) return r2;
        hipLaunchKernelGGL(k_adj_addc, dim3(std::min<int64_t>(1024, rbf::blocks_for(M, 256))),
                           dim3(256), 0, st, M, c * d, out);
        return RBF_OK;
    };
    ADJ(adj_bicgstab(S, M, pois_t, nullptr, y, w, 0.1 * S->rtol_p, std::max(S->maxit_p, 20000),
                     "rbf_adjoint_step (transposed pressure solve)"));
    hipLaunchKernelGGL(k_adj_fbar, dim3(std::min<int64_t>(1024, rbf::blocks_for(M, 256))), dim3(256),
                       0, st, M, S->p_tag, S->p_rowscale, w, 1.0 / dt, fb);
    // (17): u**_bar = u_bar + Dx^PV^T F_bar, v likewise
    ADJ(tpv(A.dxT_pv, fb, t1));
    ADJ(tpv(A.dyT_pv, fb, t2));
    adj_axpby(S, N, 1.0, ub, 1.0, t1, t1);
    adj_axpby(S, N, 1.0, vb, 1.0, t2, t2);
    // (16): r_bar = H^-T u**_bar, H^T x = x - a L^T (chi x)
    auto helm_t = [&](const double *in, double *out) -> rbf_status {
        hipLaunchKernelGGL(k_adj_split, dim3(std::min<int64_t>(1024, rbf::blocks_for(N, 256))),
                           dim3(256), 0, st, N, A.vtag, in, t3, t4);
        rbf_status r2 = tvv(A.lapT_vv, t3, out);
        if (r2 != RBF_OK) return r2;
        adj_axpby(S, N, 1.0, in, -a, out, out);
        return RBF_OK;
    };
    ADJ(adj_bicgstab(S, N, helm_t, S->h_dinv, t1, rub, S->rtol_h, std::max(S->maxit_h, 2000),
                     "rbf_adjoint_step (transposed viscous solve, u)"));
    ADJ(adj_bicgstab(S, N, helm_t, S->h_dinv, t2, rvb, S->rtol_h, std::max(S->maxit_h, 2000),
                     "rbf_adjoint_step (transposed viscous solve, v)"));
    const dim3 gN(std::min<int64_t>(1024, rbf::blocks_for(N, 256))), b256(256);
    hipLaunchKernelGGL(k_adj_split, gN, b256, 0, st, N, A.vtag, rub, ri, rw);
    hipLaunchKernelGGL(k_adj_split, gN, b256, 0, st, N, A.vtag, rvb, si, sw);
    // d/d nu: dt/2 sum chi r_bar o L (u* + u**)
    adj_axpby(S, N, 1.0, us, 1.0, uss, t1);
    adj_axpby(S, N, 1.0, vs, 1.0, vss, t2);
    ADJ(fvv(S->vv_lap, t1, t3));
    ADJ(fvv(S->vv_lap, t2, t4));
    double nq[2];
    ADJ(adj_dots<2>(S, N, AdjDots{{ri, si}, {t3, t4}}, nq));
    const double nub = 0.5 * dt * (nq[0] + nq[1]);
    // (16) right-hand side: u*_bar = chi r + a L^T (chi r); wall rows (21)
    ADJ(tvv(A.lapT_vv, ri, usb));
    adj_axpby(S, N, 1.0, ri, a, usb, usb);
    ADJ(tvv(A.lapT_vv, si, vsb));
    adj_axpby(S, N, 1.0, si, a, vsb, vsb);
    adj_axpby(S, N, 1.0, rw, 1.0, grad_bc, grad_bc);
    adj_axpby(S, N, 1.0, sw, 1.0, grad_bc + N, grad_bc + N);
    ADJ(tvp(A.dxT_vp, rw, m1));
    ADJ(tvp(A.dyT_vp, sw, m2));
    adj_axpby(S, M, dt, m1, dt, m2, m1);  // p~_j_bar
    // (14): C_j_bar, C_{j-1}_bar (the caller's C_bar arrays were copied in
    // above, so they can take C_{j-1}_bar now)
    adj_axpby(S, N, 1.5 * dt, usb, 1.0, cub, cub);
    adj_axpby(S, N, 1.5 * dt, vsb, 1.0, cvb, cvb);
    if (first) {  // C_{-1} = C_0
        adj_axpby(S, N, -0.5 * dt, usb, 1.0, cub, cub);
        adj_axpby(S, N, -0.5 * dt, vsb, 1.0, cvb, cvb);
        RBF_HIP(hipMemsetAsync(adj->cu_prev, 0, nb, st));
        RBF_HIP(hipMemsetAsync(adj->cv_prev, 0, nb, st));
    } else {
        adj_axpby(S, N, -0.5 * dt, usb, 0.0, usb, adj->cu_prev);
        adj_axpby(S, N, -0.5 * dt, vsb, 0.0, vsb, adj->cv_prev);
    }
    // (15): u_j_bar, v_j_bar
    const double *uj = fwd->u, *vj = fwd->v;
    ADJ(fvv(S->vv_dx, uj, t1));   // Dx u
    ADJ(fvv(S->vv_dy, uj, t2));   // Dy u
    ADJ(fvv(S->vv_dx, vj, t3));   // Dx v
    ADJ(fvv(S->vv_dy, vj, t4));   // Dy v
    hipLaunchKernelGGL(k_adj_adv, gN, b256, 0, st, N, uj, vj, t1, t2, t3, t4, cub, cvb, usb, vsb, qx,
                       qy, px, py);
    ADJ(tvv(A.dxT_vv, qx, t1));
    ADJ(tvv(A.dyT_vv, qy, t2));
    adj_axpby(S, N, -1.0, t1, 1.0, usb, usb);
    adj_axpby(S, N, -1.0, t2, 1.0, usb, usb);
    ADJ(tvv(A.dxT_vv, px, t1));
    ADJ(tvv(A.dyT_vv, py, t2));
    adj_axpby(S, N, -1.0, t1, 1.0, vsb, vsb);
    adj_axpby(S, N, -1.0, t2, 1.0, vsb, vsb);
#undef ADJ
    // Outputs: adjoints of the state at j.
    RBF_HIP(hipMemcpyAsync(adj->u, usb, nb, hipMemcpyDeviceToDevice, st));
    RBF_HIP(hipMemcpyAsync(adj->v, vsb, nb, hipMemcpyDeviceToDevice, st));
    RBF_HIP(hipMemcpyAsync(adj->p_tilde, m1, mb, hipMemcpyDeviceToDevice, st));
    RBF_CHECK_LAUNCH();
    RBF_HIP(hipStreamSynchronize(st));
    *dnu += nub;
    return RBF_OK;
}

// Independent instances advanced concurrently: a pool of host threads takes
// the instances in order, each thread driving rbf_step on the instance's own
// stream, so that the short kernels and host synchronisations of different
// instances overlap on the device.
extern "C" rbf_status rbf_step_batch(rbf_solver *const *solvers, int32_t count, int32_t nsteps,
                                     rbf_state *states, rbf_step_stats *stats,
                                     rbf_status *statuses, int32_t nthreads) {
    rbf::clear_error();
    RBF_ARG(count >= 0 && nsteps >= 0, "rbf_step_batch: negative count or nsteps");
    RBF_ARG(count == 0 || (solvers && states), "rbf_step_batch: NULL argument");
    for (int b = 0; b < count; ++b) {
        RBF_ARG(solvers[b], "rbf_step_batch: solver %d is NULL", b);
        for (int c = 0; c < b; ++c)
            RBF_ARG(solvers[c] != solvers[b], "rbf_step_batch: solver %d repeats solver %d", b, c);
    }
    std::vector<rbf_status> rcs(count, RBF_OK);
    std::vector<std::string> msgs(count);
    std::atomic<int> next{0};
    auto work = [&]() {
        for (;;) {
            const int b = next.fetch_add(1);
            if (b >= count) return;
            rbf_solver *S = solvers[b];
            rbf_status rc;
            if (hipSetDevice(S->device) != hipSuccess) {
                rc = RBF_E_DEVICE;
                msgs[b] = "hipSetDevice failed";
            } else {
                rc = rbf_step(S, nsteps, &states[b], stats ? &stats[b] : nullptr);
                if (rc != RBF_OK) msgs[b] = rbf_last_error();
            }
            rcs[b] = rc;
        }
    };
    const int nt = std::min<int>(count, nthreads > 0 ? nthreads : 8);
    std::vector<std::thread> pool;
    for (int t = 1; t < nt; ++t) {
        try {
            pool.emplace_back(work);
        } catch (const std::system_error &) {
            break;  // fewer threads: the remaining instances run on those started
        }
    }
    work();
    for (auto &t : pool) t.join();
    rbf_status rc = RBF_OK;
    for (int b = 0; b < count; ++b) {
        if (statuses) statuses[b] = rcs[b];
        if (rcs[b] != RBF_OK && rc == RBF_OK) {
            rc = rcs[b];
            rbf::set_error("rbf_step_batch: instance %d: %s", b, msgs[b].c_str());
        }
    }
    return rc;
}

extern "C" rbf_status rbf_solve_pressure(rbf_solver *S, const double *rhs, double *p_tilde,
                                         rbf_solve_stats *stats) {
    rbf::clear_error();
    RBF_ARG(S && rhs && p_tilde, "rbf_solve_pressure: NULL argument");
    hipLaunchKernelGGL(k_scale, dim3(rbf::blocks_for(S->M, 256)), dim3(256), 0, S->st, S->M,
                       S->p_rowscale, rhs, S->p_rhs_tmp);
    RBF_CHECK_LAUNCH();
    rbf_status rc = poisson_solve(S, S->p_rhs_tmp, p_tilde, stats);
    if (rc == RBF_OK) {
        const int nbm = nblocks_rows(S->M);
        hipLaunchKernelGGL((k_sum<1>), dim3(nbm), dim3(kThreads), 0, S->st, S->M, p_tilde,
                           S->kp.partX);
        hipLaunchKernelGGL(k_sub_mean, dim3(nbm), dim3(kThreads), 0, S->st, S->M, S->kp.partX,
                           nbm, p_tilde, p_tilde);
        RBF_CHECK_LAUNCH();
        RBF_HIP(hipStreamSynchronize(S->st));
    }
    return rc;
}

extern "C" rbf_status rbf_solver_apply_precond(rbf_solver *S, const double *y, double *z) {
    rbf::clear_error();
    RBF_ARG(S && y && z, "rbf_solver_apply_precond: NULL argument");
    if (S->aux_on) {
        RBF_ARG(!S->mixed, "rbf_solver_apply_precond: the auxiliary-lattice preconditioner of "
                           "a mixed-precision solver runs in FP32 inside its solve only");
        FgDev<double> &F = S->fg64;
        RBF_HIP(hipMemsetAsync(F.s.flag, 0, sizeof(int), S->st));
        S->lat.flag = F.s.flag;
        hipLaunchKernelGGL(k_aux_scale<double>, dim3(1024), dim3(256), 0, S->st, S->ax64, y, F.wd);
        aux_apply<double>(S, S->ax64, F, y, F.wd, F.s.one, z);
        RBF_CHECK_LAUNCH();
        RBF_HIP(hipStreamSynchronize(S->st));
        return RBF_OK;
    }
    RBF_ARG(S->pc_on, "rbf_solver_apply_precond: the solver has no pressure preconditioner");
    hipStream_t st = S->st;
    const int64_t m = S->M;
    const int nb = nblocks_rows(m);
    RBF_HIP(hipMemsetAsync(S->pk.flag, 0, sizeof(int), st));
    hipLaunchKernelGGL(k_pc_pre, dim3(nb), dim3(kThreads), 0, st, S->lat, y, m, S->pk.partGs);
    rbf_status rc = pc_apply(S);
    if (rc != RBF_OK) return rc;
    hipLaunchKernelGGL(k_pc_post, dim3(nb), dim3(kThreads), 0, st, S->lat, S->pk, y, z, m,
                       S->pk.partS, S->pk.partGs, nb);
    RBF_CHECK_LAUNCH();
    RBF_HIP(hipStreamSynchronize(st));
    return RBF_OK;
}

namespace {

// Force on a body (rbf_solver_forces): pressure part over the body's
// P-nodes, viscous part over its V-nodes; each node carries its quadrature
// weight and the unit normal pointing out of the body.  One workgroup, fixed
// summation order.
template <int KT>
__global__ void __launch_bounds__(256) k_forces(int np, const int *__restrict__ prow,
                                                const double *__restrict__ pq, int nv,
                                                const int *__restrict__ vrow,
                                                const double *__restrict__ vq, int64_t n, int k,
                                                const int *__restrict__ idx,
                                                const double *__restrict__ wdx,
                                                const double *__restrict__ wdy,
                                                const double *__restrict__ u,
                                                const double *__restrict__ v,
                                                const double *__restrict__ p, double inv_re,
                                                double *out) {
    double f[2] = {0.0, 0.0};
    for (int i = threadIdx.x; i < np; i += blockDim.x) {
        const double w = pq[3 * i], nx = pq[3 * i + 1], ny = pq[3 * i + 2];
        const double pv = p[prow[i]];
        f[0] -= w * pv * nx;
        f[1] -= w * pv * ny;
    }
    for (int i = threadIdx.x; i < nv; i += blockDim.x) {
        const double w = vq[3 * i], nx = vq[3 * i + 1], ny = vq[3 * i + 2];
        double g[2][2] = {};
        const double *ws[2] = {wdx, wdy};
        rbf::ell_row<KT, 2>(idx, ws, n, vrow[i], k, Gather2{u, v}, g);
        // g[0] = (u_x, v_x), g[1] = (u_y, v_y)
        const double sxy = g[1][0] + g[0][1];
        f[0] += w * inv_re * (2.0 * g[0][0] * nx + sxy * ny);
        f[1] += w * inv_re * (sxy * nx + 2.0 * g[1][1] * ny);
    }
    __shared__ double lds[2 * (256 / 64)];
    rbf::block_sum<2>(f, lds);
    if (threadIdx.x == 0) {
        out[0] = f[0];
        out[1] = f[1];
    }
}

// Rows of one tag ordered by angle about (cx, cy) in [0, 2 pi), with their
// periodic composite Simpson weight (4/3, 2/3 of the angle step times the
// radius, 2/3 at the first) and outward body normal (cos, sin of the
// angle).  False if the count is odd or zero.
bool ring_rule(const std::vector<double> &xy, int64_t n, const std::vector<int8_t> &tag, int t,
               double cx, double cy, double radius, std::vector<int> &rows,
               std::vector<double> &q) {
    std::vector<std::pair<double, int>> a;
    const double two_pi = 6.283185307179586476925;
    for (int64_t r = 0; r < n; ++r) {
        if (tag[r] != t) continue;
        double th = std::atan2(xy[n + r] - cy, xy[r] - cx);
        if (th < 0.0) th += two_pi;
        a.push_back({th, (int)r});
    }
    if (a.empty() || (a.size() % 2) != 0) return false;
    std::stable_sort(a.begin(), a.end(),
                     [](const std::pair<double, int> &l, const std::pair<double, int> &r) { return l.first < r.first; });
    const double d = two_pi / (double)a.size();
    rows.resize(a.size());
    q.resize(3 * a.size());
    for (size_t i = 0; i < a.size(); ++i) {
        rows[i] = a[i].second;
        q[3 * i] = ((i % 2) ? 4.0 * d / 3.0 : 2.0 * d / 3.0) * radius;
        q[3 * i + 1] = std::cos(a[i].first);
        q[3 * i + 2] = std::sin(a[i].first);
    }
    return true;
}

}  // namespace

extern "C" rbf_status rbf_solver_forces(rbf_solver *S, const rbf_grid *g, const rbf_state *state,
                                        int32_t tag, double cx, double cy, double radius,
                                        double *force) {
    rbf::clear_error();
    RBF_ARG(S && g && state && force && state->u && state->v && state->p && g->xv && g->xp &&
                g->v_tag && g->p_tag,
            "rbf_solver_forces: NULL argument");
    RBF_ARG(g->n_v == S->N && g->n_p == S->M, "rbf_solver_forces: grid sizes differ from the solver's");
    RBF_ARG(tag != 0 && std::isfinite(cx) && std::isfinite(cy) && std::isfinite(radius) && radius > 0.0,
            "rbf_solver_forces: tag must be non-zero and the circle finite");
    hipStream_t st = S->st;
    auto &F = S->forces;
    if (!F.ready || F.tag != tag || F.cx != cx || F.cy != cy || F.radius != radius) {
        const int64_t N = S->N, M = S->M;
        std::vector<double> xv(2 * N), xp(2 * M);
        std::vector<int8_t> tv(N), tp(M);
        RBF_HIP(hipMemcpyAsync(xv.data(), g->xv, 2 * N * sizeof(double), hipMemcpyDeviceToHost, st));
        RBF_HIP(hipMemcpyAsync(xp.data(), g->xp, 2 * M * sizeof(double), hipMemcpyDeviceToHost, st));
        RBF_HIP(hipMemcpyAsync(tv.data(), g->v_tag, N, hipMemcpyDeviceToHost, st));
        RBF_HIP(hipMemcpyAsync(tp.data(), g->p_tag, M, hipMemcpyDeviceToHost, st));
        RBF_HIP(hipStreamSynchronize(st));
        std::vector<int> pr, vr;
        std::vector<double> pq, vq;
        RBF_ARG(ring_rule(xp, M, tp, tag, cx, cy, radius, pr, pq) &&
                    ring_rule(xv, N, tv, tag, cx, cy, radius, vr, vq),
                "rbf_solver_forces: the body's P-nodes and V-nodes must be non-empty even counts (composite Simpson's rule)");
        if (F.cap < (int)std::max(pr.size(), vr.size())) {
            const int cap = (int)std::max(pr.size(), vr.size());
            ALLOC(F.prow, cap);
            ALLOC(F.vrow, cap);
            ALLOC(F.pq, 3 * cap);
            ALLOC(F.vq, 3 * cap);
            ALLOC(F.out, 2);
            F.cap = cap;
        }
        RBF_HIP(hipMemcpyAsync(F.prow, pr.data(), pr.size() * sizeof(int), hipMemcpyHostToDevice, st));
        RBF_HIP(hipMemcpyAsync(F.vrow, vr.data(), vr.size() * sizeof(int), hipMemcpyHostToDevice, st));
        RBF_HIP(hipMemcpyAsync(F.pq, pq.data(), pq.size() * sizeof(double), hipMemcpyHostToDevice, st));
        RBF_HIP(hipMemcpyAsync(F.vq, vq.data(), vq.size() * sizeof(double), hipMemcpyHostToDevice, st));
        RBF_HIP(hipStreamSynchronize(st));
        F.np = (int)pr.size();
        F.nv = (int)vr.size();
        F.tag = tag;
        F.cx = cx;
        F.cy = cy;
        F.radius = radius;
        F.ready = true;
    }
    if (S->k == 28)
        hipLaunchKernelGGL(k_forces<28>, dim3(1), dim3(256), 0, st, F.np, F.prow, F.pq, F.nv, F.vrow,
                           F.vq, S->N, S->k, S->idx_vv, S->vv_dx, S->vv_dy, state->u, state->v,
                           state->p, 1.0 / S->re, F.out);
    else
        hipLaunchKernelGGL(k_forces<0>, dim3(1), dim3(256), 0, st, F.np, F.prow, F.pq, F.nv, F.vrow,
                           F.vq, S->N, S->k, S->idx_vv, S->vv_dx, S->vv_dy, state->u, state->v,
                           state->p, 1.0 / S->re, F.out);
    RBF_CHECK_LAUNCH();
    RBF_HIP(hipMemcpyAsync(force, F.out, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    RBF_HIP(hipStreamSynchronize(st));
    return RBF_OK;
}

extern "C" rbf_status rbf_solver_diagnostics(rbf_solver *S, const rbf_state *state,
                                             rbf_diagnostics *out) {
    rbf::clear_error();
    RBF_ARG(S && state && out && state->u && state->v, "rbf_solver_diagnostics: NULL argument");
    hipStream_t st = S->st;
    const int nbv = (int)std::min<int64_t>(kMaxBlocks, rbf::blocks_for(S->N, kThreads));
    const int nbp = (int)std::min<int64_t>(kMaxBlocks, rbf::blocks_for(S->M, kThreads));
    double *pv = S->diag_part, *pp = S->diag_part + 3 * kMaxBlocks;
    hipLaunchKernelGGL(k_diag_v, dim3(nbv), dim3(kThreads), 0, st, S->N, state->u, state->v,
                       S->v_hmin, pv);
    if (S->k == 28)
        hipLaunchKernelGGL(k_diag_p<28>, dim3(nbp), dim3(kThreads), 0, st, S->M, S->k, S->idx_pv,
                           S->pv_dx, S->pv_dy, state->u, state->v, S->p_tag, pp);
    else
        hipLaunchKernelGGL(k_diag_p<0>, dim3(nbp), dim3(kThreads), 0, st, S->M, S->k, S->idx_pv,
                           S->pv_dx, S->pv_dy, state->u, state->v, S->p_tag, pp);
    RBF_CHECK_LAUNCH();
    std::vector<double> hv(3 * (size_t)nbv), hp(2 * (size_t)nbp);
    RBF_HIP(hipMemcpyAsync(hv.data(), pv, hv.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    RBF_HIP(hipMemcpyAsync(hp.data(), pp, hp.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    RBF_HIP(hipStreamSynchronize(st));
    auto nmax = [](double a, double b) { return (std::isnan(a) || std::isnan(b)) ? NAN : std::max(a, b); };
    double ke = 0.0, smax = 0.0, cmax = 0.0, fmx = 0.0, s2 = 0.0;
    for (int b = 0; b < nbv; ++b) {
        ke += hv[b];
        smax = nmax(smax, hv[nbv + b]);
        cmax = nmax(cmax, hv[2 * nbv + b]);
    }
    for (int b = 0; b < nbp; ++b) {
        fmx = nmax(fmx, hp[b]);
        s2 += hp[nbp + b];
    }
    out->kinetic_energy = 0.5 * ke / (double)S->N;
    out->speed_max = smax;
    out->cfl = S->dt * cmax;
    out->div_max = fmx;
    out->div_rms = S->n_interior_p > 0 ? std::sqrt(s2 / (double)S->n_interior_p) : 0.0;
    return RBF_OK;
}

extern "C" rbf_status rbf_solver_query(rbf_solver *S, rbf_solver_info *info) {
    rbf::clear_error();
    RBF_ARG(S && info, "rbf_solver_query: NULL argument");
    info->viscous_jacobi = S->h_jacobi ? 1 : 0;
    info->viscous_mixed = S->h_mixed ? 1 : 0;
    info->lattice_precond = S->pc_on ? 1 : 0;
    info->jacobi_bound = S->h_bound;
    info->aux_precond = S->aux_on ? 1 : 0;
    info->aux_smooth_weight = S->aux_on ? S->ax64.w2 : 0.0;
    info->aux_cells = S->aux_K;
    return RBF_OK;
}

extern "C" rbf_status rbf_solver_profile(rbf_solver *S, int32_t sample_every, double *avg_ms,
                                         int64_t *count) {
    rbf::clear_error();
    RBF_ARG(S, "rbf_solver_profile: NULL solver");
    for (int q = 0; q < RBF_PROF_N; ++q) {
        if (avg_ms) avg_ms[q] = S->prof_count[q] ? S->prof_ms[q] / (double)S->prof_count[q] : 0.0;
        if (count) count[q] = S->prof_count[q];
    }
    if (sample_every >= 0) {
        if (sample_every > 0 && S->prof_ev[0].empty()) {
            for (int q = 0; q < RBF_PROF_N; ++q) {
                S->prof_ev[q].resize(2 * rbf_solver::kProfPairs, nullptr);
                for (auto &e : S->prof_ev[q]) RBF_HIP(hipEventCreate(&e));
            }
        }
        S->prof_every = sample_every;
        S->prof_launches = 0;
        for (int q = 0; q < RBF_PROF_N; ++q) {
            S->prof_count[q] = 0;
            S->prof_ms[q] = 0.0;
        }
    }
    return RBF_OK;
}

extern "C" void rbf_solver_destroy(rbf_solver *S) {
    if (!S) return;
    if (S->st) hipStreamSynchronize(S->st);
    for (auto &v : S->prof_ev)
        for (hipEvent_t e : v)
            if (e) hipEventDestroy(e);
    for (void *p : S->allocs) hipFree(p);
    if (S->hflag) hipHostFree(S->hflag);
    if (S->hred) hipHostFree(S->hred);
    delete S;
}
