// Reverse-mode derivative of one step of Sec. 3 (eqs. (14)-(21)), kernels.
// Included by solver.hip inside its anonymous namespace.
//
// The adjoint of the step transposes its stages in reverse order (u_bar:
// adjoint of u, and so on; chi: interior indicator; G = D^VP, D = D^PV):
//   u**_bar = u_{j+1}_bar,  p~_bar -= dt (Gx^T u_bar + Gy^T v_bar)      (20)
//   rhs_bar = S w, (A_s + u1 c 1^T)^T w = p~_bar - mean(p~_bar)         (18)
//   F_bar = chi_P rhs_bar / dt,  u**_bar += Dx^T F_bar, v likewise      (17)
//   r_bar = H^-T u**_bar (both components)                              (16)
//   nu_bar += dt/2 sum chi r_bar o L (u* + u**)   (H and (I + aL) in nu)
//   u*_bar = chi r_bar + a L^T (chi r_bar);  u_bc_bar += (1 - chi) r_bar;
//   p~_j_bar = dt (Gx^T ((1 - chi) r_u_bar) + Gy^T ((1 - chi) r_v_bar)) (21)
//   C_j_bar = 3/2 dt u*_bar + (C_j as the next step's C_{j-1})_bar,
//   C_{j-1}_bar = -1/2 dt u*_bar (folded into C_j_bar at j = 0)         (14)
//   u_j_bar = u*_bar - Dx u o Cu_bar - Dx^T(u o Cu_bar) - Dy^T(v o Cu_bar)
//             - Dx v o Cv_bar, v_j_bar likewise                         (15)
// Here S is the row scale of the stored Poisson rows A_s = S A0 and
// u1 = S chi: the transpose of the zero-mean bordered solve of the forward
// step is a solve with (A_s + u1 c 1^T)^T followed by the row scale.
#pragma once

// out = alpha a + beta b (elementwise; b may alias out).
__global__ void k_adj_axpby(int64_t n, double alpha, const double *__restrict__ a, double beta,
                            const double *b, double *out) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = alpha * a[i] + beta * b[i];
}

// Split r by the V-node tags: ri = chi r (interior), rw = (1 - chi) r.
__global__ void k_adj_split(int64_t n, const int8_t *__restrict__ tag, const double *__restrict__ r,
                            double *ri, double *rw) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const bool wall = tag[i] != 0;
        ri[i] = wall ? 0.0 : r[i];
        rw[i] = wall ? r[i] : 0.0;
    }
}

// out = a o b (elementwise product).
__global__ void k_adj_mul(int64_t n, const double *__restrict__ a, const double *__restrict__ b,
                          double *out) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = a[i] * b[i];
}

// F_bar = chi_P s o w / dt (row scale s, interior P rows only).
__global__ void k_adj_fbar(int64_t m, const int8_t *__restrict__ ptag, const double *__restrict__ s,
                           const double *__restrict__ w, double inv_dt, double *fb) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x)
        fb[i] = (ptag[i] == 0) ? s[i] * w[i] * inv_dt : 0.0;
}

// Advection adjoint, pointwise part: with cu_b, cv_b the adjoints of C_j,
//   ub -= (Dx u) cu_b + (Dx v) cv_b,  vb -= (Dy u) cu_b + (Dy v) cv_b,
// and the gather inputs of the transposed products
//   qx = u cu_b, qy = v cu_b (for u_bar), px = u cv_b, py = v cv_b (for v_bar).
__global__ void k_adj_adv(int64_t n, const double *__restrict__ u, const double *__restrict__ v,
                          const double *__restrict__ dxu, const double *__restrict__ dyu,
                          const double *__restrict__ dxv, const double *__restrict__ dyv,
                          const double *__restrict__ cub, const double *__restrict__ cvb,
                          double *ub, double *vb, double *qx, double *qy, double *px, double *py) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double a = cub[i], b = cvb[i];
        ub[i] -= dxu[i] * a + dxv[i] * b;
        vb[i] -= dyu[i] * a + dyv[i] * b;
        qx[i] = u[i] * a;
        qy[i] = v[i] * a;
        px[i] = u[i] * b;
        py[i] = v[i] * b;
    }
}

// Up to four dot products (x_q, y_q), or sums when y_q is null.
struct AdjDots {
    const double *x[4];
    const double *y[4];
};

// Block partial sums of NQ dot products of d (row q at q * kMaxBlocks).
template <int NQ>
__global__ void __launch_bounds__(kThreads) k_adj_dots(int64_t n, AdjDots d, double *part) {
    double acc[NQ] = {};
    for (int64_t i = blockIdx.x * (int64_t)kThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kThreads) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) acc[q] += d.x[q][i] * (d.y[q] ? d.y[q][i] : 1.0);
    }
    __shared__ double lds[NQ * (kThreads / 64)];
    rbf::block_sum<NQ>(acc, lds);
    if (threadIdx.x == 0)
        for (int q = 0; q < NQ; ++q) part[(int64_t)q * kMaxBlocks + blockIdx.x] = acc[q];
}

// z += c (elementwise constant).
__global__ void k_adj_addc(int64_t n, double c, double *z) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        z[i] += c;
}

// tag[r] = 1 for the wall rows in list (the array is zero beforehand).
__global__ void k_adj_wallmask(int64_t nwall, const int *__restrict__ list, int8_t *tag) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < nwall) tag[list[i]] = 1;
}
