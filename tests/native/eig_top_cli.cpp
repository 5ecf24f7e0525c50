// Command-line driver of the host eigensolver (csrc/eig_top.h) for the CPU tests: reads
// int32 n and n*n float64 (row-major) from stdin, writes float64 lambda and the n
// components of the unit eigenvector to stdout; exit status 0, or 3 when the solver
// reports failure.
#include <cstdint>
#include <cstdio>
#include <vector>

#include "../../paper_1207_5558_amd/csrc/eig_top.h"

int main() {
    int32_t n = 0;
    if (fread(&n, sizeof n, 1, stdin) != 1 || n < 0 || n > 4096) return 2;
    std::vector<double> A((size_t)n * n);
    if (n > 0 && fread(A.data(), sizeof(double), A.size(), stdin) != A.size()) return 2;
    double lam = 0.0;
    std::vector<double> x;
    if (slsht::sym_top_eigenpair(A, n, &lam, x) != 0) return 3;
    fwrite(&lam, sizeof lam, 1, stdout);
    fwrite(x.data(), sizeof(double), x.size(), stdout);
    return 0;
}
