// Host driver for rbf_build_nodes under AddressSanitizer and
// UndefinedBehaviorSanitizer (built by tests/test_host_sanitizers.py).
// Usage: nodes_driver <kind> <K> <jitter> <seed> <out.bin>
// Runs the two-call pattern, the argument checks, and writes
// n_v, n_p (int64), xv, xp, p_normal (double), v_tag, p_tag (int8) to out.bin.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "rbffd.h"

int main(int argc, char **argv) {
    if (argc != 6) return 2;
    const int kind = std::atoi(argv[1]), K = std::atoi(argv[2]);
    const double jitter = std::atof(argv[3]);
    const uint64_t seed = std::strtoull(argv[4], nullptr, 10);
    int64_t nv = -1, np = -1;
    if (rbf_build_nodes(kind, K, jitter, seed, &nv, nullptr, nullptr, &np, nullptr, nullptr,
                        nullptr) != RBF_OK)
        return 3;
    std::vector<double> xv(2 * nv), xp(2 * np), pn(2 * np);
    std::vector<int8_t> vt(nv), pt(np);
    if (rbf_build_nodes(kind, K, jitter, seed, &nv, xv.data(), vt.data(), &np, xp.data(),
                        pt.data(), pn.data()) != RBF_OK)
        return 4;
    // Argument checks: each must fail with RBF_E_ARG and touch nothing.
    int64_t a = 0, b = 0;
    if (rbf_build_nodes(7, K, jitter, seed, &a, nullptr, nullptr, &b, nullptr, nullptr, nullptr) !=
        RBF_E_ARG)
        return 5;
    if (rbf_build_nodes(kind, K, 0.5, seed, &a, nullptr, nullptr, &b, nullptr, nullptr, nullptr) !=
        RBF_E_ARG)
        return 6;
    if (rbf_build_nodes(kind, K, jitter, seed, &a, xv.data(), nullptr, &b, nullptr, nullptr,
                        nullptr) != RBF_E_ARG)
        return 7;
    if (rbf_build_nodes(0, 1, jitter, seed, &a, nullptr, nullptr, &b, nullptr, nullptr, nullptr) !=
        RBF_E_ARG)
        return 8;
    if (rbf_last_error()[0] == '\0') return 9;
    FILE *f = std::fopen(argv[5], "wb");
    if (!f) return 10;
    std::fwrite(&nv, sizeof nv, 1, f);
    std::fwrite(&np, sizeof np, 1, f);
    std::fwrite(xv.data(), sizeof(double), xv.size(), f);
    std::fwrite(xp.data(), sizeof(double), xp.size(), f);
    std::fwrite(pn.data(), sizeof(double), pn.size(), f);
    std::fwrite(vt.data(), 1, vt.size(), f);
    std::fwrite(pt.data(), 1, pt.size(), f);
    std::fclose(f);
    return 0;
}
