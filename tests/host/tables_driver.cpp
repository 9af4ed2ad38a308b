// Prints the host-side plan and tables of the library for one L and delta*kappa, so the
// CPU tests can check them against independent references.  Built by the tests with g++.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "hub_tables.hpp"

int main(int argc, char** argv) {
    if (argc != 3 && argc != 4) return 2;
    const int L = std::atoi(argv[1]);
    const double dk = std::atof(argv[2]);
    const double dmu = argc == 4 ? std::atof(argv[3]) : 0.0;
    hub::FftPlan plan{};
    if (!hub::make_plan(L, &plan)) {
        std::printf("noplan\n");
        return 0;
    }
    std::printf("plan %d", plan.nst);
    for (int q = 0; q < plan.nst; ++q) std::printf(" %d", plan.radix[q]);
    std::printf("\n");
    std::printf("pos");
    for (int k = 0; k < L; ++k) std::printf(" %d", hub::digit_reversed_position(plan, k));
    std::printf("\n");
    std::vector<double> roots, etab;
    hub::build_tables(plan, dk, dmu, roots, etab);
    for (int m = 0; m < L; ++m) std::printf("root %.17g %.17g\n", roots[2 * m], roots[2 * m + 1]);
    for (int p = 0; p < L * L; ++p)
        std::printf("e %.17g %.17g %.17g\n", etab[4 * p], etab[4 * p + 1], etab[4 * p + 2]);
    return 0;
}
