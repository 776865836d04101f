// rbf_ell_apply: y = D x for one slot-major ELL operator (eq. (10) applied
// to a vector), FP64 or FP32-stored; plus the FP64 -> FP32 cast helper.
//
// One thread per row.  For a fixed stencil width all index and weight loads
// of the row are issued (non-temporal: the operator streams through once)
// before the gathers of x, which hit in the caches because stencil
// neighbours are close in memory; blocks are remapped so that every XCD
// works on one contiguous range of rows (its L2 then holds that range of x).
#include "common.h"

namespace {

template <class T>
__device__ __forceinline__ T fma_t(T a, T b, T c);
template <>
__device__ __forceinline__ double fma_t<double>(double a, double b, double c) { return fma(a, b, c); }
template <>
__device__ __forceinline__ float fma_t<float>(float a, float b, float c) { return fmaf(a, b, c); }

template <class T, int KT>
__global__ void __launch_bounds__(256) k_ell_apply(int64_t rows, int k, const int *__restrict__ idx,
                                                   const T *__restrict__ w, const T *__restrict__ x,
                                                   T *__restrict__ y) {
    const uint32_t lb = rbf::xcd_block(blockIdx.x, gridDim.x);
    const int64_t r = (int64_t)lb * blockDim.x + threadIdx.x;
    if (r >= rows) return;
    T acc = T(0);
    if constexpr (KT > 0) {
        int jj[KT];
        T ww[KT];
#pragma unroll
        for (int s = 0; s < KT; ++s) jj[s] = rbf::ld_stream(idx + (int64_t)s * rows + r);
#pragma unroll
        for (int s = 0; s < KT; ++s) ww[s] = rbf::ld_stream(w + (int64_t)s * rows + r);
#pragma unroll
        for (int s = 0; s < KT; ++s) acc = fma_t<T>(ww[s], x[jj[s]], acc);
    } else {
#pragma unroll 4
        for (int s = 0; s < k; ++s)
            acc = fma_t<T>(rbf::ld_stream(w + (int64_t)s * rows + r),
                           x[rbf::ld_stream(idx + (int64_t)s * rows + r)], acc);
    }
    y[r] = acc;
}

__global__ void k_cast_f32(const double *__restrict__ a, float *__restrict__ b, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        b[i] = (float)a[i];
}

}  // namespace

extern "C" rbf_status rbf_ell_apply(int64_t rows, int32_t k, const int32_t *idx, const void *w,
                                    const void *x, void *y, int32_t dtype, rbf_stream st_) {
    rbf::clear_error();
    RBF_ARG(rows >= 0 && rows < (int64_t)1 << 31, "rbf_ell_apply: rows out of range");
    RBF_ARG(k >= 1 && k <= 64, "rbf_ell_apply: k must be in [1, 64]");
    RBF_ARG(dtype == 0 || dtype == 1, "rbf_ell_apply: dtype must be 0 (FP64) or 1 (FP32)");
    if (rows == 0) return RBF_OK;
    RBF_ARG(idx && w && x && y, "rbf_ell_apply: NULL pointer");
    hipStream_t st = rbf::as_stream(st_);
    const dim3 grid(rbf::blocks_for(rows, 256)), block(256);
    if (dtype == 0) {
        auto W = static_cast<const double *>(w);
        auto X = static_cast<const double *>(x);
        auto Y = static_cast<double *>(y);
        if (k == 28) hipLaunchKernelGGL((k_ell_apply<double, 28>), grid, block, 0, st, rows, k, idx, W, X, Y);
        else hipLaunchKernelGGL((k_ell_apply<double, 0>), grid, block, 0, st, rows, k, idx, W, X, Y);
    } else {
        auto W = static_cast<const float *>(w);
        auto X = static_cast<const float *>(x);
        auto Y = static_cast<float *>(y);
        if (k == 28) hipLaunchKernelGGL((k_ell_apply<float, 28>), grid, block, 0, st, rows, k, idx, W, X, Y);
        else hipLaunchKernelGGL((k_ell_apply<float, 0>), grid, block, 0, st, rows, k, idx, W, X, Y);
    }
    RBF_CHECK_LAUNCH();
    return RBF_OK;
}

extern "C" rbf_status rbf_cast_f32(const double *src, float *dst, int64_t n, rbf_stream st_) {
    rbf::clear_error();
    RBF_ARG(n >= 0, "rbf_cast_f32: n < 0");
    if (n == 0) return RBF_OK;
    RBF_ARG(src && dst, "rbf_cast_f32: NULL pointer");
    hipLaunchKernelGGL(k_cast_f32, dim3(1024), dim3(256), 0, rbf::as_stream(st_), src, dst, n);
    RBF_CHECK_LAUNCH();
    return RBF_OK;
}
