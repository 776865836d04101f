// rbf_build_nodes: seeded staggered node sets (host code).
//
// Stand-in for the DistMesh grids of Sec. 3: P-nodes on the vertices of a
// triangulation, V-nodes on the edge midpoints (kinds 0 and 2).  Randomness is SplitMix64
// (Steele, Lea & Flood 2014) used as a counter-based generator.  Every
// floating-point expression is evaluated with one rounding per operation
// (this file is compiled with -ffp-contract=off), so the coordinates are a
// fixed function of (kind, K, jitter, seed).
#include <cmath>
#include <cstdint>

#include "common.h"

namespace {

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kMix1 = 0xBF58476D1CE4E5B9ull;
constexpr uint64_t kMix2 = 0x94D049BB133111EBull;
constexpr uint64_t kStreamV = 0, kStreamP = 1;
constexpr double kSqrtHalf = 0.7071067811865476;  // 1/sqrt(2), nearest double

uint64_t splitmix64(uint64_t seed, uint64_t counter) {
    uint64_t z = seed + (counter + 1) * kGamma;
    z = (z ^ (z >> 30)) * kMix1;
    z = (z ^ (z >> 27)) * kMix2;
    return z ^ (z >> 31);
}

double uniform01(uint64_t seed, uint64_t stream, uint64_t c) {
    return static_cast<double>(splitmix64(seed, (stream << 40) | c) >> 11) * 0x1.0p-53;
}

// Jitter offsets of node n: draws 2n (x) and 2n+1 (y) of the stream.
void jitter(uint64_t seed, uint64_t stream, uint64_t n, double amp, double &ox, double &oy) {
    double ux = uniform01(seed, stream, 2 * n);
    double uy = uniform01(seed, stream, 2 * n + 1);
    ox = (2.0 * ux - 1.0) * amp;
    oy = (2.0 * uy - 1.0) * amp;
}

void cavity(int K, double jit, uint64_t seed, double *xv, int8_t *vtag, double *xp,
            int8_t *ptag, double *pn, int64_t N, int64_t M) {
    const double h = 1.0 / K;
    const double amp = jit * h;
    const int n1 = K + 1;
    for (int j = 0; j <= K; ++j) {
        for (int i = 0; i <= K; ++i) {
            const int64_t v = (int64_t)j * n1 + i;
            const bool interior = i > 0 && i < K && j > 0 && j < K;
            double ox, oy;
            jitter(seed, kStreamP, (uint64_t)v, amp, ox, oy);
            double px = (i == K) ? 1.0 : (double)i * h;
            double py = (j == K) ? 1.0 : (double)j * h;
            if (interior) {
                px = px + ox;
                py = py + oy;
            }
            xp[v] = px;
            xp[M + v] = py;
            ptag[v] = interior ? 0 : 1;
            double nx = (i == 0) ? -1.0 : (i == K ? 1.0 : 0.0);
            double ny = (j == 0) ? -1.0 : (j == K ? 1.0 : 0.0);
            if (nx != 0.0 && ny != 0.0) {
                nx = nx * kSqrtHalf;
                ny = ny * kSqrtHalf;
            }
            pn[v] = nx;
            pn[M + v] = ny;
        }
    }
    int64_t e = 0;
    auto emit = [&](int64_t a, int64_t b) {
        const double ax = xp[a], ay = xp[M + a], bx = xp[b], by = xp[M + b];
        const double vx = (ax + bx) * 0.5, vy = (ay + by) * 0.5;
        xv[e] = vx;
        xv[N + e] = vy;
        const bool both = ptag[a] != 0 && ptag[b] != 0;
        const bool wall = both && ((ax == bx && (ax == 0.0 || ax == 1.0)) ||
                                   (ay == by && (ay == 0.0 || ay == 1.0)));
        vtag[e] = wall ? (vy == 1.0 ? 2 : 1) : 0;
        ++e;
    };
    for (int j = 0; j <= K; ++j) {
        for (int i = 0; i <= K; ++i) {
            const int64_t v = (int64_t)j * n1 + i;
            if (i < K) emit(v, v + 1);
            if (j < K) emit(v, v + n1);
            if (i < K && j < K) {
                if ((i + j) % 2 == 0) emit(v, v + n1 + 1);
                else emit(v + 1, v + n1);
            }
        }
    }
}

void square(int K, double jit, uint64_t seed, double *xv, int8_t *vtag, double *xp,
            int8_t *ptag, double *pn, int64_t n) {
    const double h = 1.0 / K;
    const double amp = jit * h;
    for (int j = 0; j < K; ++j) {
        for (int i = 0; i < K; ++i) {
            const int64_t v = (int64_t)j * K + i;
            double ox, oy;
            jitter(seed, kStreamV, (uint64_t)v, amp, ox, oy);
            xv[v] = ((double)i + 0.5) * h + ox;
            xv[n + v] = ((double)j + 0.5) * h + oy;
            jitter(seed, kStreamP, (uint64_t)v, amp, ox, oy);
            xp[v] = (double)i * h + ox;
            xp[n + v] = (double)j * h + oy;
            vtag[v] = 0;
            ptag[v] = 0;
            pn[v] = 0.0;
            pn[n + v] = 0.0;
        }
    }
}

// Near-equilateral cavity (kind 2).  Row j of the P-grid (j = 0..R,
// y_j = j/R) holds n_j nodes; hex_key(j, i) is node i's unjittered x.
int hex_rows(int K) { return (int)std::floor(2.0 * (double)K / std::sqrt(3.0) + 0.5); }

int hex_row_len(int K, int R, int j) {
    if (j == 0 || j == R || j % 2 == 0) return K + 1;
    return K + 2;
}

double hex_key(int K, int R, int j, int i) {
    const double h = 1.0 / K;
    const int n = hex_row_len(K, R, j);
    if (i == 0) return 0.0;
    if (i == n - 1) return 1.0;
    if (j == 0 || j == R || j % 2 == 0) return (double)i * h;
    return ((double)(i - 1) + 0.5) * h;
}

void hex_counts(int K, int64_t &N, int64_t &M) {
    const int R = hex_rows(K);
    N = 0;
    M = 0;
    for (int j = 0; j <= R; ++j) {
        const int64_t n = hex_row_len(K, R, j);
        M += n;
        N += n - 1;  // horizontal edges of the row
        if (j < R) N += n + hex_row_len(K, R, j + 1) - 1;  // strip edges
    }
}

void hex_cavity(int K, double jit, uint64_t seed, double *xv, int8_t *vtag, double *xp,
                int8_t *ptag, double *pn, int64_t N, int64_t M) {
    const double h = 1.0 / K;
    const double amp = jit * h;
    const int R = hex_rows(K);
    int64_t v = 0;
    for (int j = 0; j <= R; ++j) {
        const int n = hex_row_len(K, R, j);
        const double y = (j == R) ? 1.0 : (double)j / (double)R;
        for (int i = 0; i < n; ++i, ++v) {
            const double x = hex_key(K, R, j, i);
            const bool wall = j == 0 || j == R || i == 0 || i == n - 1;
            const double dw = std::fmin(std::fmin(x, y), std::fmin(1.0 - x, 1.0 - y));
            double px = x, py = y;
            if (!wall && dw >= 1.5 * h) {
                double ox, oy;
                jitter(seed, kStreamP, (uint64_t)v, amp, ox, oy);
                px = px + ox;
                py = py + oy;
            }
            xp[v] = px;
            xp[M + v] = py;
            ptag[v] = wall ? 1 : 0;
            double nx = 0.0, ny = 0.0;
            if (wall) {
                nx = (px == 0.0) ? -1.0 : (px == 1.0 ? 1.0 : 0.0);
                ny = (py == 0.0) ? -1.0 : (py == 1.0 ? 1.0 : 0.0);
                if (nx != 0.0 && ny != 0.0) {
                    nx = nx * kSqrtHalf;
                    ny = ny * kSqrtHalf;
                }
            }
            pn[v] = nx;
            pn[M + v] = ny;
        }
    }
    int64_t e = 0;
    auto emit = [&](int64_t a, int64_t b) {
        const double ax = xp[a], ay = xp[M + a], bx = xp[b], by = xp[M + b];
        const double vx = (ax + bx) * 0.5, vy = (ay + by) * 0.5;
        xv[e] = vx;
        xv[N + e] = vy;
        const bool both = ptag[a] != 0 && ptag[b] != 0;
        const bool wall = both && ((ax == bx && (ax == 0.0 || ax == 1.0)) ||
                                   (ay == by && (ay == 0.0 || ay == 1.0)));
        vtag[e] = wall ? (vy == 1.0 ? 2 : 1) : 0;
        ++e;
    };
    int64_t a0 = 0;
    for (int j = 0; j <= R; ++j) {
        const int na = hex_row_len(K, R, j);
        for (int i = 0; i + 1 < na; ++i) emit(a0 + i, a0 + i + 1);
        if (j == R) break;
        const int nb = hex_row_len(K, R, j + 1);
        const int64_t b0 = a0 + na;
        int ia = 0, ib = 0;
        emit(a0, b0);
        while (ia < na - 1 || ib < nb - 1) {
            if (ia == na - 1) ++ib;
            else if (ib == nb - 1) ++ia;
            else if (hex_key(K, R, j, ia + 1) <= hex_key(K, R, j + 1, ib + 1)) ++ia;
            else ++ib;
            emit(a0 + ia, b0 + ib);
        }
        a0 = b0;
    }
}

}  // namespace

extern "C" rbf_status rbf_build_nodes(int32_t kind, int32_t K, double jitter_frac, uint64_t seed,
                                      int64_t *n_v, double *xv, int8_t *v_tag, int64_t *n_p,
                                      double *xp, int8_t *p_tag, double *p_normal) {
    rbf::clear_error();
    RBF_ARG(n_v && n_p, "rbf_build_nodes: n_v and n_p must not be NULL");
    RBF_ARG(jitter_frac >= 0.0 && jitter_frac <= 0.45, "rbf_build_nodes: jitter must be in [0, 0.45]");
    int64_t N, M;
    if (kind == 0) {
        RBF_ARG(K >= 2 && K <= 20000, "rbf_build_nodes: cavity needs 2 <= K <= 20000");
        N = 3ll * K * K + 2ll * K;
        M = (int64_t)(K + 1) * (K + 1);
    } else if (kind == 1) {
        RBF_ARG(K >= 1 && K <= 30000, "rbf_build_nodes: square needs 1 <= K <= 30000");
        N = M = (int64_t)K * K;
    } else if (kind == 2) {
        RBF_ARG(K >= 2 && K <= 20000, "rbf_build_nodes: near-equilateral cavity needs 2 <= K <= 20000");
        RBF_ARG(jitter_frac <= 0.4, "rbf_build_nodes: kind 2 needs jitter <= 0.4 (rows stay apart)");
        hex_counts(K, N, M);
    } else {
        RBF_ARG(false, "rbf_build_nodes: unknown kind %d", kind);
    }
    *n_v = N;
    *n_p = M;
    const bool none = !xv && !v_tag && !xp && !p_tag && !p_normal;
    const bool all = xv && v_tag && xp && p_tag && p_normal;
    RBF_ARG(none || all, "rbf_build_nodes: pass all arrays or none");
    if (none) return RBF_OK;
    if (kind == 0) cavity(K, jitter_frac, seed, xv, v_tag, xp, p_tag, p_normal, N, M);
    else if (kind == 1) square(K, jitter_frac, seed, xv, v_tag, xp, p_tag, p_normal, N);
    else hex_cavity(K, jitter_frac, seed, xv, v_tag, xp, p_tag, p_normal, N, M);
    return RBF_OK;
}
