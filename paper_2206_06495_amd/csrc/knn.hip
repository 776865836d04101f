// rbf_knn: exact k-nearest-neighbour stencils on the GPU.
//
// Sec. 2.2 builds row r of D^(alpha,beta) from the n nearest beta-nodes of
// the alpha-node r.  The stencil is defined as the first k beta-nodes in the
// order of the key (d^2, index), with d^2 = dx*dx + dy*dy evaluated with
// separately rounded products (this file is compiled with
// -ffp-contract=off), so the result is unique even on lattices with ties.
//
// Method: a uniform cell grid over the source bounding box (counting sort of
// the sources by cell), then one thread per query searching square rings of
// cells outward.  The thread keeps its best k candidates as a sorted list in
// registers (fully unrolled insertion, static indices) and stops once the
// k-th best squared distance is strictly below the squared distance to every
// cell not yet visited.
#include <algorithm>
#include <climits>
#include <cmath>
#include <mutex>

#include "common.h"

namespace {

struct Grid {
    double x0, y0, c, inv_c;
    int gx, gy;
};

__device__ __forceinline__ bool key_less(double d, int i, double bd, int bi) {
    return d < bd || (d == bd && i < bi);
}

__device__ __forceinline__ int cell_coord(double v, double v0, double inv_c, int g) {
    double t = floor((v - v0) * inv_c);
    int c = (t < 0.0) ? 0 : (t >= (double)g ? g - 1 : (int)t);
    return c;
}

// Per-block bounding box of n points plus a non-finite flag: part[5 b + 0..3]
// = min x, max x, min y, max y over the finite points, part[5 b + 4] = 1 if
// any coordinate is NaN or infinite (fmin/fmax alone would skip a NaN).
__global__ void k_bbox_partial(const double *__restrict__ x, int64_t n, double *__restrict__ part) {
    __shared__ double lds[5 * 16];
    double v[5] = {INFINITY, -INFINITY, INFINITY, -INFINITY, 0.0};
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        double px = x[i], py = x[n + i];
        v[0] = fmin(v[0], px);
        v[1] = fmax(v[1], px);
        v[2] = fmin(v[2], py);
        v[3] = fmax(v[3], py);
        if (!isfinite(px) || !isfinite(py)) v[4] = 1.0;
    }
    for (int off = 32; off >= 1; off >>= 1) {
        v[0] = fmin(v[0], __shfl_xor(v[0], off, 64));
        v[1] = fmax(v[1], __shfl_xor(v[1], off, 64));
        v[2] = fmin(v[2], __shfl_xor(v[2], off, 64));
        v[3] = fmax(v[3], __shfl_xor(v[3], off, 64));
        v[4] = fmax(v[4], __shfl_xor(v[4], off, 64));
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if (lane == 0)
        for (int q = 0; q < 5; ++q) lds[q * 16 + wid] = v[q];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < nw; ++w) {
            v[0] = fmin(v[0], lds[w]);
            v[1] = fmax(v[1], lds[16 + w]);
            v[2] = fmin(v[2], lds[32 + w]);
            v[3] = fmax(v[3], lds[48 + w]);
            v[4] = fmax(v[4], lds[64 + w]);
        }
        for (int q = 0; q < 5; ++q) part[blockIdx.x * 5 + q] = v[q];
    }
}

__global__ void k_zero_i32(int *__restrict__ a, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        a[i] = 0;
}

__global__ void k_cell_count(const double *__restrict__ x, int64_t n, Grid g,
                             int *__restrict__ cell, int *__restrict__ count) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    int cx = cell_coord(x[i], g.x0, g.inv_c, g.gx);
    int cy = cell_coord(x[n + i], g.y0, g.inv_c, g.gy);
    int c = cy * g.gx + cx;
    cell[i] = c;
    atomicAdd(&count[c], 1);
}

// Exclusive scan of count[0..n) into start[0..n], one block of 1024 threads.
__global__ void k_scan(const int *__restrict__ count, int64_t n, int *__restrict__ start) {
    __shared__ int lds[1024];
    const int t = threadIdx.x;
    const int64_t chunk = (n + 1023) / 1024;
    const int64_t a = t * chunk, b = (a + chunk < n) ? a + chunk : n;
    int s = 0;
    for (int64_t i = a; i < b; ++i) s += count[i];
    lds[t] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        int v = (t >= off) ? lds[t - off] : 0;
        __syncthreads();
        lds[t] += v;
        __syncthreads();
    }
    int run = lds[t] - s;
    for (int64_t i = a; i < b; ++i) {
        start[i] = run;
        run += count[i];
    }
    if (t == 1023) start[n] = lds[1023];
}

__global__ void k_scatter(const double *__restrict__ x, int64_t n, const int *__restrict__ cell,
                          const int *__restrict__ start, int *__restrict__ fill,
                          double *__restrict__ sx, double *__restrict__ sy, int *__restrict__ sid) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    int c = cell[i];
    int pos = start[c] + atomicAdd(&fill[c], 1);
    sx[pos] = x[i];
    sy[pos] = x[n + i];
    sid[pos] = (int)i;
}

template <int KMAX>
__global__ void __launch_bounds__(128) k_query(const double *__restrict__ xq, int64_t nq, int k,
                                               Grid g, const int *__restrict__ start,
                                               const double *__restrict__ sx,
                                               const double *__restrict__ sy,
                                               const int *__restrict__ sid,
                                               int *__restrict__ idx) {
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= nq) return;
    const double qx = xq[q], qy = xq[nq + q];
    const int cx = cell_coord(qx, g.x0, g.inv_c, g.gx);
    const int cy = cell_coord(qy, g.y0, g.inv_c, g.gy);
    double bd[KMAX];
    int bi[KMAX];
#pragma unroll
    for (int s = 0; s < KMAX; ++s) {
        bd[s] = INFINITY;
        bi[s] = INT_MAX;
    }
    double thr_d = INFINITY;
    int thr_i = INT_MAX;
    const int rmax = max(max(cx, g.gx - 1 - cx), max(cy, g.gy - 1 - cy));
    for (int r = 0; r <= rmax; ++r) {
        const int ylo = cy - r, yhi = cy + r;
        for (int iy = max(ylo, 0); iy <= min(yhi, g.gy - 1); ++iy) {
            const bool full_row = (iy == ylo) || (iy == yhi);
            const int step = full_row ? 1 : 2 * r;
            for (int ix = cx - r; ix <= cx + r; ix += (step > 0 ? step : 1)) {
                if (ix < 0 || ix >= g.gx) continue;
                const int c = iy * g.gx + ix;
                const int pe = start[c + 1];
                for (int p = start[c]; p < pe; ++p) {
                    const double dx = sx[p] - qx;
                    const double dy = sy[p] - qy;
                    const double d2 = dx * dx + dy * dy;
                    const int id = sid[p];
                    if (!key_less(d2, id, thr_d, thr_i)) continue;
                    // Sorted insertion; the former last entry drops out.
#pragma unroll
                    for (int s = KMAX - 1; s > 0; --s) {
                        const bool before_prev = key_less(d2, id, bd[s - 1], bi[s - 1]);
                        const bool before_cur = key_less(d2, id, bd[s], bi[s]);
                        if (before_prev) {
                            bd[s] = bd[s - 1];
                            bi[s] = bi[s - 1];
                        } else if (before_cur) {
                            bd[s] = d2;
                            bi[s] = id;
                        }
                    }
                    if (key_less(d2, id, bd[0], bi[0])) {
                        bd[0] = d2;
                        bi[0] = id;
                    }
#pragma unroll
                    for (int s = 0; s < KMAX; ++s)
                        if (s == k - 1) {
                            thr_d = bd[s];
                            thr_i = bi[s];
                        }
                }
                if (step == 0) break;
            }
        }
        if (thr_d == INFINITY) continue;  // fewer than k candidates so far
        // Distance from the query to the nearest cell outside the block.
        double bound = INFINITY;
        if (cx - r > 0) bound = fmin(bound, qx - (g.x0 + (double)(cx - r) * g.c));
        if (cx + r < g.gx - 1) bound = fmin(bound, (g.x0 + (double)(cx + r + 1) * g.c) - qx);
        if (cy - r > 0) bound = fmin(bound, qy - (g.y0 + (double)(cy - r) * g.c));
        if (cy + r < g.gy - 1) bound = fmin(bound, (g.y0 + (double)(cy + r + 1) * g.c) - qy);
        if (bound == INFINITY) break;
        bound -= 1e-9 * g.c;  // margin for the rounding of cell assignment
        if (bound > 0.0 && thr_d < bound * bound) break;
    }
#pragma unroll
    for (int s = 0; s < KMAX; ++s)
        if (s < k) idx[(int64_t)s * nq + q] = bi[s];
}

// Device buffers of one kNN call besides its inputs and output.
struct KnnScratch {
    double *part;  // [2][kBboxBlocks][5] bounding-box partials (sources, queries)
    int *cell, *count, *start, *fill, *sid;
    double *sx, *sy;
};

constexpr int kBboxBlocks = 256;

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Bytes of the cell-grid buffers for ns sources and ncell cells.
size_t grid_bytes(int64_t ns, int64_t ncell) {
    return 2 * align256(ns * sizeof(int)) + 2 * align256(ns * sizeof(double)) +
           2 * align256(ncell * sizeof(int)) + align256((ncell + 1) * sizeof(int));
}

// Lays the cell-grid buffers out in [base, base + grid_bytes).
void carve_grid(char *base, int64_t ns, int64_t ncell, KnnScratch &s) {
    auto take = [&](size_t b) { char *p = base; base += align256(b); return p; };
    s.cell = (int *)take(ns * sizeof(int));
    s.sid = (int *)take(ns * sizeof(int));
    s.sx = (double *)take(ns * sizeof(double));
    s.sy = (double *)take(ns * sizeof(double));
    s.count = (int *)take(ncell * sizeof(int));
    s.fill = (int *)take(ncell * sizeof(int));
    s.start = (int *)take((ncell + 1) * sizeof(int));
}

rbf_status knn_check_args(const double *xq, int64_t nq, const double *xs, int64_t ns, int32_t k,
                          int32_t *idx) {
    RBF_ARG(k >= 1 && k <= 64, "rbf_knn: k must be in [1, 64] (got %d)", k);
    RBF_ARG(ns >= 1 && k <= ns, "rbf_knn: need 1 <= k <= ns (k=%d, ns=%lld)", k, (long long)ns);
    RBF_ARG(nq >= 0 && nq < INT_MAX && ns < INT_MAX, "rbf_knn: sizes out of range");
    RBF_ARG(xs && (nq == 0 || (xq && idx)), "rbf_knn: NULL pointer");
    return RBF_OK;
}

// Bounding box of the sources and finiteness of both node sets (one stream
// synchronisation); fills the cell grid g and its cell count.
rbf_status knn_grid(const double *xq, int64_t nq, const double *xs, int64_t ns, double *part,
                    hipStream_t st, Grid &g, int64_t &ncell) {
    hipLaunchKernelGGL(k_bbox_partial, dim3(kBboxBlocks), dim3(1024), 0, st, xs, ns, part);
    RBF_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_bbox_partial, dim3(kBboxBlocks), dim3(1024), 0, st, xq, nq,
                       part + 5 * kBboxBlocks);
    RBF_CHECK_LAUNCH();
    double hpart[2 * kBboxBlocks * 5];
    RBF_HIP(hipMemcpyAsync(hpart, part, sizeof(hpart), hipMemcpyDeviceToHost, st));
    RBF_HIP(hipStreamSynchronize(st));
    double bb[4] = {INFINITY, -INFINITY, INFINITY, -INFINITY};
    bool bad_src = false, bad_query = false;
    for (int b = 0; b < kBboxBlocks; ++b) {
        bb[0] = fmin(bb[0], hpart[5 * b]);
        bb[1] = fmax(bb[1], hpart[5 * b + 1]);
        bb[2] = fmin(bb[2], hpart[5 * b + 2]);
        bb[3] = fmax(bb[3], hpart[5 * b + 3]);
        bad_src = bad_src || hpart[5 * b + 4] != 0.0;
        bad_query = bad_query || hpart[5 * (kBboxBlocks + b) + 4] != 0.0;
    }
    RBF_ARG(!bad_src && std::isfinite(bb[0]) && std::isfinite(bb[1]) && std::isfinite(bb[2]) &&
                std::isfinite(bb[3]),
            "rbf_knn: non-finite source coordinates");
    RBF_ARG(!bad_query, "rbf_knn: non-finite query coordinates");
    const double ex = bb[1] - bb[0], ey = bb[3] - bb[2];
    double c = sqrt(fmax(ex * ey, 0.0) * 2.0 / (double)ns);
    c = fmax(c, fmax(ex, ey) / 4096.0);
    if (!(c > 0.0)) c = 1.0;
    g.x0 = bb[0];
    g.y0 = bb[2];
    g.c = c;
    g.inv_c = 1.0 / c;
    g.gx = (int)(ex * g.inv_c) + 1;
    g.gy = (int)(ey * g.inv_c) + 1;
    ncell = (int64_t)g.gx * g.gy;
    return RBF_OK;
}

// Counting sort of the sources by cell, then the queries; synchronises.
rbf_status knn_search(const double *xq, int64_t nq, const double *xs, int64_t ns, int32_t k,
                      int32_t *idx, hipStream_t st, const Grid &g, int64_t ncell,
                      const KnnScratch &s) {
    const uint32_t zb = (uint32_t)std::min<int64_t>(rbf::blocks_for(ncell, 256), 1024);
    hipLaunchKernelGGL(k_zero_i32, dim3(zb), dim3(256), 0, st, s.count, ncell);
    hipLaunchKernelGGL(k_zero_i32, dim3(zb), dim3(256), 0, st, s.fill, ncell);
    hipLaunchKernelGGL(k_cell_count, dim3(rbf::blocks_for(ns, 256)), dim3(256), 0, st, xs, ns, g,
                       s.cell, s.count);
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, s.count, ncell, s.start);
    hipLaunchKernelGGL(k_scatter, dim3(rbf::blocks_for(ns, 256)), dim3(256), 0, st, xs, ns,
                       s.cell, s.start, s.fill, s.sx, s.sy, s.sid);
    if (k <= 32)
        hipLaunchKernelGGL(k_query<32>, dim3(rbf::blocks_for(nq, 128)), dim3(128), 0, st, xq, nq,
                           k, g, s.start, s.sx, s.sy, s.sid, idx);
    else
        hipLaunchKernelGGL(k_query<64>, dim3(rbf::blocks_for(nq, 128)), dim3(128), 0, st, xq, nq,
                           k, g, s.start, s.sx, s.sy, s.sid, idx);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        rbf::set_error("rbf_knn: %s", hipGetErrorString(e));
        return RBF_E_DEVICE;
    }
    return RBF_OK;
}

}  // namespace

extern "C" rbf_status rbf_knn(const double *xq, int64_t nq, const double *xs, int64_t ns,
                              int32_t k, int32_t *idx, rbf_stream st_) {
    rbf::clear_error();
    rbf_status rc = knn_check_args(xq, nq, xs, ns, k, idx);
    if (rc != RBF_OK || nq == 0) return rc;
    hipStream_t st = rbf::as_stream(st_);
    KnnScratch s{};
    RBF_HIP(hipMalloc(&s.part, 2 * kBboxBlocks * 5 * sizeof(double)));
    Grid g;
    int64_t ncell = 0;
    rc = knn_grid(xq, nq, xs, ns, s.part, st, g, ncell);
    char *base = nullptr;
    if (rc == RBF_OK) {
        if (hipMalloc(&base, grid_bytes(ns, ncell)) != hipSuccess) {
            rbf::set_error("rbf_knn: device allocation failed");
            rc = RBF_E_NOMEM;
        } else {
            carve_grid(base, ns, ncell, s);
            rc = knn_search(xq, nq, xs, ns, k, idx, st, g, ncell, s);
        }
    }
    hipFree(base);
    hipFree(s.part);
    return rc;
}

// ------------------------------------------------------ no-allocation form --
// A fixed per-device scratch array for callers that cannot allocate device
// memory.  In host code `scratch` names a host-side stand-in, not device
// memory: its device address is taken once per device with
// hipGetSymbolAddress and only that address is used.
namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch_addr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first
// call on that device, with that device current).
rbf_status scratch_address(char **out) {
    int dev = -1;
    RBF_HIP(hipGetDevice(&dev));
    RBF_ARG(dev >= 0 && dev < kMaxDevices, "rbf_knn_noalloc: device ordinal %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[dev]) {
        void *p = nullptr;
        RBF_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        RBF_ARG(p != nullptr, "rbf_knn_noalloc: no device address for the scratch array");
        g_scratch_addr[dev] = static_cast<char *>(p);
    }
    *out = g_scratch_addr[dev];
    return RBF_OK;
}

}  // namespace

extern "C" rbf_status rbf_knn_noalloc(const double *xq, int64_t nq, const double *xs, int64_t ns,
                                      int32_t k, int32_t *idx, rbf_stream st_) {
    rbf::clear_error();
    rbf_status rc = knn_check_args(xq, nq, xs, ns, k, idx);
    if (rc != RBF_OK || nq == 0) return rc;
    const size_t part_bytes = align256(2 * kBboxBlocks * 5 * sizeof(double));
    // The grid has at most ns/2 + 8193 cells (cell edge >= sqrt(2 area/ns)
    // and >= the longer box side / 4096), so this bound needs no device work.
    RBF_ARG(part_bytes + grid_bytes(ns, ns / 2 + 8194) <= kScratchBytes,
            "rbf_knn_noalloc: %lld sources exceed the %zu-byte scratch array (at most about "
            "%lld sources)",
            (long long)ns, kScratchBytes,
            (long long)((kScratchBytes - part_bytes - 8194 * 12 - 2048) / 30));
    char *base = nullptr;
    rc = scratch_address(&base);
    if (rc != RBF_OK) return rc;
    hipStream_t st = rbf::as_stream(st_);
    KnnScratch s{};
    s.part = reinterpret_cast<double *>(base);
    Grid g;
    int64_t ncell = 0;
    rc = knn_grid(xq, nq, xs, ns, s.part, st, g, ncell);
    if (rc != RBF_OK) return rc;
    RBF_ARG(part_bytes + grid_bytes(ns, ncell) <= kScratchBytes,
            "rbf_knn_noalloc: cell grid of %lld cells exceeds the scratch array",
            (long long)ncell);
    carve_grid(base + part_bytes, ns, ncell, s);
    return knn_search(xq, nq, xs, ns, k, idx, st, g, ncell, s);
}
