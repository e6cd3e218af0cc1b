// Reads "m k" and then the m diagonal and m-1 off-diagonal entries of a
// symmetric tridiagonal matrix from stdin; prints the k smallest eigenvalues
// and their eigenvectors (one line each) as computed by tridiag_smallest.
#include <cstdio>
#include <vector>

#include "tridiag.h"

int main()
{
    int m = 0, k = 0;
    if (std::scanf("%d %d", &m, &k) != 2 || m <= 0 || k <= 0) return 2;
    std::vector<double> d(m), e(m > 1 ? m - 1 : 1), vals(k), vecs((size_t)k * m);
    for (int i = 0; i < m; ++i)
        if (std::scanf("%lf", &d[i]) != 1) return 2;
    for (int i = 0; i + 1 < m; ++i)
        if (std::scanf("%lf", &e[i]) != 1) return 2;
    const int got = vpp::tridiag_smallest(m, d.data(), e.data(), k, vals.data(), vecs.data());
    std::printf("%d\n", got);
    for (int t = 0; t < got; ++t) std::printf("%.17g\n", vals[t]);
    for (int t = 0; t < got; ++t) {
        for (int j = 0; j < m; ++j) std::printf("%.17g ", vecs[(size_t)t * m + j]);
        std::printf("\n");
    }
    return 0;
}
