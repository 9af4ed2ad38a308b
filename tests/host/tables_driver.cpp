// Prints the host-side plan and tables of the library for one L and delta*kappa (or, with
// "poly X DEG", the exponential's polynomial on [-X, X]), so the CPU tests can check them
// against independent references.  Built by the tests with g++.
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "hub_tables.hpp"

int main(int argc, char** argv) {
    if (argc == 4 && std::string(argv[1]) == "poly") {      // poly X DEG: the stencil's polynomial
        double a0 = 0.0, r[9] = {};
        const int deg = std::atoi(argv[3]);
        const double err = hub::exp_poly_ratios(std::atof(argv[2]), deg, &a0, r);
        std::printf("err %.17g\na0 %.17g\nratios", err, a0);
        for (int k = 1; k <= deg; ++k) std::printf(" %.17g", r[k]);
        std::printf("\n");
        return 0;
    }
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
