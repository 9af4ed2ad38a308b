// Host-side plan and tables (plain C++: no HIP types, so host tests can build them alone).
#pragma once

#include <vector>

namespace hub {

constexpr int kMaxStages = 12;     // L <= 1024 has at most 10 prime factors

// Mixed-radix factorisation of L used by every in-LDS transform.  Stage q works
// on blocks of length len[q] = L / (radix[0] * ... * radix[q-1]).
struct FftPlan {
    int L;
    int nst;
    int radix[kMaxStages];
    int len[kMaxStages];
};

bool make_plan(int L, FftPlan* plan);

// Position of momentum index k (0 <= k < L) after the in-place forward transform:
// the transform leaves frequencies in mixed-radix digit-reversed order.
int digit_reversed_position(const FftPlan& plan, int k);

// Host-side FP64 tables.
//   roots[m]   = e^{-2 pi i m / L}, m = 0..L-1, angles from the integer m (exact), as (re, im)
//   etab[p]    = (c, Re sf, Im sf, 0) / L^2 at transform position p = p1*L + p2, where
//                k = (k1, k2) is the momentum stored at p, f = 1 + e^{-i k1} + e^{-i k2},
//                c = cosh(dk |f|), s = sinh(dk |f|)/|f| (-> dk at |f| = 0), sf = s*f,
//                all times e^{delta mu}.
void build_tables(const FftPlan& plan, double delta_kappa, double delta_mu, std::vector<double>& roots,
                  std::vector<double>& etab);

}  // namespace hub
