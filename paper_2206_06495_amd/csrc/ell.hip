// rbf_ell_apply: y = D x for one slot-major ELL operator (eq. (10) applied
// to a vector), FP64 or FP32-stored; plus the FP64 -> FP32 cast helper.
// rbf_ell_transpose / rbf_ell_transpose_weights / rbf_ell_apply_transpose:
// z = D^T y through a column structure built once and weights permuted into
// column order, in a fixed summation order (no floating-point atomics).
//
// One thread per row.  For a fixed stencil width all index and weight loads
// of the row are issued (non-temporal: the operator streams through once)
// before the gathers of x, which hit in the caches because stencil
// neighbours are close in memory; blocks are remapped so that every XCD
// works on one contiguous range of rows (its L2 then holds that range of x).
#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>

#include "common.h"

namespace {

template <class T>
__device__ __forceinline__ T fma_t(T a, T b, T c);
template <>
__device__ __forceinline__ double fma_t<double>(double a, double b, double c) { return fma(a, b, c); }
template <>
__device__ __forceinline__ float fma_t<float>(float a, float b, float c) { return fmaf(a, b, c); }

// Launch shape of the fixed-width product (chosen by rbf_ell_autotune):
// XCD: blocks remapped to one contiguous row range per XCD; NT: operator
// loads non-temporal.  The row's summation order is the same in every
// shape, so every shape gives the same bits.
template <class T, bool NT>
__device__ __forceinline__ T ell_load(const T *p) {
    if constexpr (NT) return rbf::ld_stream(p);
    else return *p;
}

template <class T, int KT, bool XCD = true, bool NT = true>
__global__ void __launch_bounds__(512) k_ell_apply(int64_t rows, int k, const int *__restrict__ idx,
                                                   const T *__restrict__ w, const T *__restrict__ x,
                                                   T *__restrict__ y) {
    const uint32_t lb = XCD ? rbf::xcd_block(blockIdx.x, gridDim.x) : blockIdx.x;
    const int64_t r = (int64_t)lb * blockDim.x + threadIdx.x;
    if (r >= rows) return;
    T acc = T(0);
    if constexpr (KT > 0) {
        int jj[KT];
        T ww[KT];
#pragma unroll
        for (int s = 0; s < KT; ++s) jj[s] = ell_load<int, NT>(idx + (int64_t)s * rows + r);
#pragma unroll
        for (int s = 0; s < KT; ++s) ww[s] = ell_load<T, NT>(w + (int64_t)s * rows + r);
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

// ---------------------------------------------------------- transpose --
// Column counts: cnt[c + 1] = number of ELL entries (s, r) with
// idx[s][r] == c (cnt[0] stays 0).  Entries outside [0, ncols) are not
// counted; the lowest such ELL position goes to *bad.
__global__ void k_tr_count(int64_t nnz, const int *__restrict__ idx, int64_t ncols,
                           unsigned long long *cnt, unsigned long long *bad) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int c = idx[e];
        if (c < 0 || (int64_t)c >= ncols) atomicMin(bad, (unsigned long long)e);
        else atomicAdd(cnt + c + 1, 1ull);
    }
}

// Longest column: max over c of cnt[c + 1] into *mx.
__global__ void k_tr_maxlen(int64_t ncols, const int64_t *__restrict__ cnt, unsigned long long *mx) {
    unsigned long long m = 0;
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < ncols;
         c += (int64_t)gridDim.x * blockDim.x)
        m = max(m, (unsigned long long)cnt[c + 1]);
    atomicMax(mx, m);
}

// In-place inclusive prefix sum of a[0..n) in one workgroup of kScanT
// threads: chunks of kScanT * kScanV values, each thread summing kScanV
// consecutive values, a Hillis-Steele scan of the thread totals in LDS, and
// a carry across chunks.  Set-up work (one pass over the columns).
constexpr int kScanT = 1024, kScanV = 8;
__global__ void __launch_bounds__(kScanT) k_tr_scan(int64_t n, int64_t *a) {
    __shared__ int64_t tot[2][kScanT];
    int64_t carry = 0;
    for (int64_t base = 0; base < n; base += (int64_t)kScanT * kScanV) {
        const int64_t i0 = base + (int64_t)threadIdx.x * kScanV;
        int64_t v[kScanV], run = 0;
#pragma unroll
        for (int j = 0; j < kScanV; ++j) {
            v[j] = (i0 + j < n) ? a[i0 + j] : 0;
            run += v[j];
            v[j] = run;
        }
        int cur = 0;
        tot[cur][threadIdx.x] = run;
        __syncthreads();
        for (int off = 1; off < kScanT; off <<= 1) {
            const int64_t t = tot[cur][threadIdx.x] +
                              (threadIdx.x >= off ? tot[cur][threadIdx.x - off] : 0);
            tot[cur ^ 1][threadIdx.x] = t;
            cur ^= 1;
            __syncthreads();
        }
        const int64_t before = carry + (threadIdx.x ? tot[cur][threadIdx.x - 1] : 0);
#pragma unroll
        for (int j = 0; j < kScanV; ++j)
            if (i0 + j < n) a[i0 + j] = before + v[j];
        carry += tot[cur][kScanT - 1];
        __syncthreads();
    }
}

// Scatter: entry (s, r) of column c goes to colptr[c] + (arrival order);
// the order inside a column is fixed afterwards by k_tr_sort.
__global__ void k_tr_fill(int64_t rows, int64_t nnz, const int *__restrict__ idx,
                          const int64_t *__restrict__ colptr, int *cursor, int *src, int *slot) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int c = idx[e];
        const int64_t pos = colptr[c] + atomicAdd(cursor + c, 1);
        src[pos] = (int)(e % rows);
        slot[pos] = (int)(e / rows);
    }
}

// Per column: insertion sort of its entries by (source row, slot).  Columns
// hold about k entries (at most kMaxColumn, checked before launch), so one
// thread per column.
constexpr int64_t kMaxColumn = 4096;
__global__ void k_tr_sort(int64_t ncols, const int64_t *__restrict__ colptr, int *src, int *slot) {
    const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (c >= ncols) return;
    const int64_t b = colptr[c], e = colptr[c + 1];
    for (int64_t i = b + 1; i < e; ++i) {
        const int r = src[i], s = slot[i];
        int64_t j = i - 1;
        while (j >= b && (src[j] > r || (src[j] == r && slot[j] > s))) {
            src[j + 1] = src[j];
            slot[j + 1] = slot[j];
            --j;
        }
        src[j + 1] = r;
        slot[j + 1] = s;
    }
}

// Weights in column order: wt[e] = w[slot[e]][src[e]] (one gather per
// weight array, so that products read them contiguously).
template <class T>
__global__ void k_tr_weights(int64_t rows, int64_t nnz, const int *__restrict__ src,
                             const int *__restrict__ slot, const T *__restrict__ w,
                             T *__restrict__ wt) {
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz;
         e += (int64_t)gridDim.x * blockDim.x)
        wt[e] = w[(int64_t)slot[e] * rows + src[e]];
}

// z_c = sum of wt[e] * y[src[e]] over the entries e of column c.  One
// wavefront per 64 consecutive columns, whose entries are one contiguous
// range: the wave walks that range in chunks of kTrChunk entries with
// coalesced loads (lane l takes entries l, l + 64, ...), writes the
// products wt[e] * y[src[e]] to LDS, and then every lane adds the products
// of its own column in entry order.  The order of the additions is fixed
// by the column structure alone, so results are reproducible bit for bit.
constexpr int kTrChunk = 512;
constexpr int kTrWaves = 4;
template <class T>
__global__ void __launch_bounds__(64 * kTrWaves) k_ell_apply_t(int64_t ncols,
                                                               const int64_t *__restrict__ colptr,
                                                               const int *__restrict__ src,
                                                               const T *__restrict__ wt,
                                                               const T *__restrict__ y,
                                                               T *__restrict__ z) {
    __shared__ T prod[kTrWaves][kTrChunk];
    const uint32_t lb = rbf::xcd_block(blockIdx.x, gridDim.x);
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t c0 = ((int64_t)lb * kTrWaves + wv) * 64;
    if (c0 >= ncols) return;  // whole waves leave together
    const int64_t c = c0 + lane;
    const int64_t cend = min(c0 + 64, ncols);
    const int64_t E0 = colptr[c0], E1 = colptr[cend];
    const int64_t b = (c < ncols) ? colptr[c] : E1, e = (c < ncols) ? colptr[c + 1] : E1;
    T *pw = prod[wv];
    T acc = T(0);
    for (int64_t ch = E0; ch < E1; ch += kTrChunk) {
        const int64_t n = min((int64_t)kTrChunk, E1 - ch);
#pragma unroll 4
        for (int t = lane; t < n; t += 64) pw[t] = wt[ch + t] * y[src[ch + t]];
        __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): this wave's LDS writes are done
        __builtin_amdgcn_wave_barrier();
        const int64_t lo = max(b, ch), hi = min(e, ch + n);
        for (int64_t i = lo; i < hi; ++i) acc += pw[i - ch];
        __builtin_amdgcn_wave_barrier();
    }
    if (c < ncols) z[c] = acc;
}

}  // namespace

namespace {

// Launch shapes of the 28-wide product: block size x XCD remap x operator
// load kind.  Shape 0 is the default (256 threads, remap, non-temporal).
constexpr int kEllShapes = 16;
struct EllShape {
    int block;
    bool xcd, nt;
};
constexpr EllShape kShapes[kEllShapes] = {
    {256, true, true},   {64, true, true},   {128, true, true},   {512, true, true},
    {256, false, true},  {64, false, true},  {128, false, true},  {512, false, true},
    {256, true, false},  {64, true, false},  {128, true, false},  {512, true, false},
    {256, false, false}, {64, false, false}, {128, false, false}, {512, false, false}};

// Tuned shapes, per (dtype, k, rows) (process-wide).
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int64_t>, int> g_tuned;

int tuned_shape(int dtype, int k, int64_t rows) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(std::make_tuple(dtype, k, rows));
    return it == g_tuned.end() ? 0 : it->second;
}

template <class T>
void launch_ell_28(int shape, int64_t rows, const int32_t *idx, const T *W, const T *X, T *Y,
                   hipStream_t st) {
    const EllShape sh = kShapes[shape];
    const dim3 grid(rbf::blocks_for(rows, sh.block)), block(sh.block);
#define RBF_ELL(XC, NTL) \
    hipLaunchKernelGGL((k_ell_apply<T, 28, XC, NTL>), grid, block, 0, st, rows, 28, idx, W, X, Y)
    if (sh.xcd && sh.nt) RBF_ELL(true, true);
    else if (!sh.xcd && sh.nt) RBF_ELL(false, true);
    else if (sh.xcd) RBF_ELL(true, false);
    else RBF_ELL(false, false);
#undef RBF_ELL
}

}  // namespace

extern "C" rbf_status rbf_ell_autotune(int64_t rows, int32_t k, const int32_t *idx, const void *w,
                                       const void *x, void *y, int32_t dtype, int32_t reps,
                                       int32_t *shape, float *ms, rbf_stream st_) {
    rbf::clear_error();
    RBF_ARG(rows > 0 && rows < (int64_t)1 << 31, "rbf_ell_autotune: rows out of range");
    RBF_ARG(k >= 1 && k <= 64, "rbf_ell_autotune: k must be in [1, 64]");
    RBF_ARG(dtype == 0 || dtype == 1, "rbf_ell_autotune: dtype must be 0 (FP64) or 1 (FP32)");
    RBF_ARG(reps >= 1 && reps <= 10000, "rbf_ell_autotune: reps must be in [1, 10000]");
    RBF_ARG(idx && w && x && y && shape, "rbf_ell_autotune: NULL pointer");
    hipStream_t st = rbf::as_stream(st_);
    if (k != 28) {  // one shape for the generic width
        *shape = 0;
        if (ms)
            for (int v = 0; v < kEllShapes; ++v) ms[v] = (v == 0) ? 0.0f : -1.0f;
        return RBF_OK;
    }
    hipEvent_t e0, e1;
    RBF_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        hipEventDestroy(e0);
        rbf::set_error("rbf_ell_autotune: event creation failed");
        return RBF_E_DEVICE;
    }
    float best = INFINITY;
    int bi = 0;
    hipError_t err = hipSuccess;
    for (int v = 0; v < kEllShapes && err == hipSuccess; ++v) {
        auto run = [&]() {
            if (dtype == 0)
                launch_ell_28<double>(v, rows, idx, static_cast<const double *>(w),
                                      static_cast<const double *>(x), static_cast<double *>(y), st);
            else
                launch_ell_28<float>(v, rows, idx, static_cast<const float *>(w),
                                     static_cast<const float *>(x), static_cast<float *>(y), st);
        };
        run();  // warm-up
        err = hipEventRecord(e0, st);
        for (int r = 0; r < reps && err == hipSuccess; ++r) run();
        if (err == hipSuccess) err = hipGetLastError();
        if (err == hipSuccess) err = hipEventRecord(e1, st);
        if (err == hipSuccess) err = hipEventSynchronize(e1);
        float t = 0.0f;
        if (err == hipSuccess) err = hipEventElapsedTime(&t, e0, e1);
        t /= (float)reps;
        if (ms) ms[v] = t;
        if (t < best) {  // strict: ties keep the earlier (default-first) shape
            best = t;
            bi = v;
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (err != hipSuccess) {
        rbf::set_error("rbf_ell_autotune: %s", hipGetErrorString(err));
        return RBF_E_DEVICE;
    }
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tuned[std::make_tuple((int)dtype, (int)k, rows)] = bi;
    }
    *shape = bi;
    return RBF_OK;
}

extern "C" rbf_status rbf_ell_apply(int64_t rows, int32_t k, const int32_t *idx, const void *w,
                                    const void *x, void *y, int32_t dtype, rbf_stream st_) {
    rbf::clear_error();
    RBF_ARG(rows >= 0 && rows < (int64_t)1 << 31, "rbf_ell_apply: rows out of range");
    RBF_ARG(k >= 1 && k <= 64, "rbf_ell_apply: k must be in [1, 64]");
    RBF_ARG(dtype == 0 || dtype == 1, "rbf_ell_apply: dtype must be 0 (FP64) or 1 (FP32)");
    if (rows == 0) return RBF_OK;
    RBF_ARG(idx && w && x && y, "rbf_ell_apply: NULL pointer");
    hipStream_t st = rbf::as_stream(st_);
    if (k == 28) {
        const int shape = tuned_shape(dtype, k, rows);
        if (dtype == 0)
            launch_ell_28<double>(shape, rows, idx, static_cast<const double *>(w),
                                  static_cast<const double *>(x), static_cast<double *>(y), st);
        else
            launch_ell_28<float>(shape, rows, idx, static_cast<const float *>(w),
                                 static_cast<const float *>(x), static_cast<float *>(y), st);
        RBF_CHECK_LAUNCH();
        return RBF_OK;
    }
    const dim3 grid(rbf::blocks_for(rows, 256)), block(256);
    if (dtype == 0) {
        auto W = static_cast<const double *>(w);
        auto X = static_cast<const double *>(x);
        auto Y = static_cast<double *>(y);
        hipLaunchKernelGGL((k_ell_apply<double, 0>), grid, block, 0, st, rows, k, idx, W, X, Y);
    } else {
        auto W = static_cast<const float *>(w);
        auto X = static_cast<const float *>(x);
        auto Y = static_cast<float *>(y);
        hipLaunchKernelGGL((k_ell_apply<float, 0>), grid, block, 0, st, rows, k, idx, W, X, Y);
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

extern "C" rbf_status rbf_ell_transpose(int64_t rows, int32_t k, const int32_t *idx, int64_t ncols,
                                        int64_t *colptr, int32_t *src, int32_t *slot,
                                        int64_t *bad_entry, rbf_stream st_) {
    rbf::clear_error();
    RBF_ARG(rows >= 0 && k >= 1 && k <= 64 && rows * k < ((int64_t)1 << 31),
            "rbf_ell_transpose: rows * k must be below 2^31 and k in [1, 64]");
    RBF_ARG(ncols >= 0 && ncols < ((int64_t)1 << 31), "rbf_ell_transpose: ncols out of range");
    RBF_ARG(bad_entry, "rbf_ell_transpose: bad_entry is NULL");
    *bad_entry = -1;
    RBF_ARG(colptr, "rbf_ell_transpose: colptr is NULL");
    hipStream_t st = rbf::as_stream(st_);
    const int64_t nnz = rows * k;
    RBF_HIP(hipMemsetAsync(colptr, 0, (size_t)(ncols + 1) * sizeof(int64_t), st));
    if (nnz == 0) return RBF_OK;
    RBF_ARG(idx && src && slot, "rbf_ell_transpose: NULL pointer");
    // Workspace: the bad-entry marker and one arrival counter per column.
    void *ws = nullptr;
    const size_t wsb = 256 + (size_t)(ncols > 0 ? ncols : 1) * sizeof(int);
    RBF_HIP(hipMalloc(&ws, wsb));
    auto *bad = static_cast<unsigned long long *>(ws);
    int *cursor = reinterpret_cast<int *>(static_cast<char *>(ws) + 256);
    rbf_status rc = RBF_OK;
    unsigned long long hbad = ~0ull;
    auto run = [&]() -> rbf_status {
        RBF_HIP(hipMemsetAsync(ws, 0xff, 256, st));
        RBF_HIP(hipMemsetAsync(cursor, 0, wsb - 256, st));
        const uint32_t ge = std::min<uint32_t>(rbf::blocks_for(nnz, 256), 8192u);
        hipLaunchKernelGGL(k_tr_count, dim3(ge), dim3(256), 0, st, nnz, idx, ncols,
                           reinterpret_cast<unsigned long long *>(colptr), bad);
        RBF_CHECK_LAUNCH();
        unsigned long long *mx = bad + 1, hm[2] = {~0ull, 0};
        RBF_HIP(hipMemsetAsync(mx, 0, sizeof(*mx), st));
        if (ncols > 0)
            hipLaunchKernelGGL(k_tr_maxlen, dim3(std::min<uint32_t>(rbf::blocks_for(ncols, 256), 1024u)),
                               dim3(256), 0, st, ncols, colptr, mx);
        RBF_CHECK_LAUNCH();
        RBF_HIP(hipMemcpyAsync(hm, bad, sizeof(hm), hipMemcpyDeviceToHost, st));
        RBF_HIP(hipStreamSynchronize(st));
        hbad = hm[0];
        if (hbad == ~0ull && hm[1] > (unsigned long long)kMaxColumn) {
            rbf::set_error("rbf_ell_transpose: a column holds %llu entries (at most %lld)", hm[1],
                           (long long)kMaxColumn);
            return RBF_E_ARG;
        }
        if (hbad != ~0ull) {
            *bad_entry = (int64_t)hbad;
            rbf::set_error("rbf_ell_transpose: idx entry %lld (slot %lld, row %lld) is outside [0, %lld)",
                           (long long)hbad, (long long)(hbad / rows), (long long)(hbad % rows),
                           (long long)ncols);
            return RBF_E_ARG;
        }
        hipLaunchKernelGGL(k_tr_scan, dim3(1), dim3(kScanT), 0, st, ncols + 1, colptr);
        hipLaunchKernelGGL(k_tr_fill, dim3(ge), dim3(256), 0, st, (int64_t)rows, nnz, idx, colptr,
                           cursor, src, slot);
        if (ncols > 0)
            hipLaunchKernelGGL(k_tr_sort, dim3(rbf::blocks_for(ncols, 256)), dim3(256), 0, st,
                               ncols, colptr, src, slot);
        RBF_CHECK_LAUNCH();
        RBF_HIP(hipStreamSynchronize(st));
        return RBF_OK;
    };
    rc = run();
    if (rc != RBF_OK) (void)hipStreamSynchronize(st);
    const hipError_t fe = hipFree(ws);
    if (rc == RBF_OK && fe != hipSuccess) {
        rbf::set_error("rbf_ell_transpose: hipFree failed: %s", hipGetErrorString(fe));
        rc = RBF_E_DEVICE;
    }
    return rc;
}

extern "C" rbf_status rbf_ell_transpose_weights(int64_t rows, int32_t k, const int32_t *src,
                                                const int32_t *slot, const void *w, void *wt,
                                                int32_t dtype, rbf_stream st_) {
    rbf::clear_error();
    RBF_ARG(rows >= 0 && k >= 1 && k <= 64 && rows * k < ((int64_t)1 << 31),
            "rbf_ell_transpose_weights: rows * k must be below 2^31 and k in [1, 64]");
    RBF_ARG(dtype == 0 || dtype == 1, "rbf_ell_transpose_weights: dtype must be 0 (FP64) or 1 (FP32)");
    const int64_t nnz = rows * k;
    if (nnz == 0) return RBF_OK;
    RBF_ARG(src && slot && w && wt, "rbf_ell_transpose_weights: NULL pointer");
    hipStream_t st = rbf::as_stream(st_);
    const dim3 grid(std::min<uint32_t>(rbf::blocks_for(nnz, 256), 8192u)), block(256);
    if (dtype == 0)
        hipLaunchKernelGGL(k_tr_weights<double>, grid, block, 0, st, rows, nnz, src, slot,
                           static_cast<const double *>(w), static_cast<double *>(wt));
    else
        hipLaunchKernelGGL(k_tr_weights<float>, grid, block, 0, st, rows, nnz, src, slot,
                           static_cast<const float *>(w), static_cast<float *>(wt));
    RBF_CHECK_LAUNCH();
    return RBF_OK;
}

extern "C" rbf_status rbf_ell_apply_transpose(int64_t ncols, const int64_t *colptr,
                                              const int32_t *src, const void *wt, const void *y,
                                              void *z, int32_t dtype, rbf_stream st_) {
    rbf::clear_error();
    RBF_ARG(ncols >= 0 && ncols < ((int64_t)1 << 31), "rbf_ell_apply_transpose: ncols out of range");
    RBF_ARG(dtype == 0 || dtype == 1, "rbf_ell_apply_transpose: dtype must be 0 (FP64) or 1 (FP32)");
    if (ncols == 0) return RBF_OK;
    RBF_ARG(colptr && z, "rbf_ell_apply_transpose: NULL pointer");
    hipStream_t st = rbf::as_stream(st_);
    const dim3 grid(rbf::blocks_for(ncols, 64 * kTrWaves)), block(64 * kTrWaves);
    if (dtype == 0)
        hipLaunchKernelGGL(k_ell_apply_t<double>, grid, block, 0, st, ncols, colptr, src,
                           static_cast<const double *>(wt), static_cast<const double *>(y),
                           static_cast<double *>(z));
    else
        hipLaunchKernelGGL(k_ell_apply_t<float>, grid, block, 0, st, ncols, colptr, src,
                           static_cast<const float *>(wt), static_cast<const float *>(y),
                           static_cast<float *>(z));
    RBF_CHECK_LAUNCH();
    return RBF_OK;
}
