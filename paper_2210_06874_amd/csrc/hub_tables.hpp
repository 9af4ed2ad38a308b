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

// A polynomial p(z) = sum_{k<=deg} a_k z^k close to e^z on z in [-x, x], for applying
// exp(delta kappa K) as p(delta kappa K): the spectrum of delta kappa K lies in [-x, x] with
// x = 3 |delta kappa| (K's eigenvalues are +-|f(k)|, |f| <= 3), so the operator error in the
// 2-norm is at most max |p(z) - e^z| over [-x, x].  p is the Chebyshev series of e^z on [-x, x]
// truncated at degree deg (coefficients 2 I_j(x), modified Bessel functions, evaluated by their
// power series in long double; its error is about 2 I_{deg+1}(x) ~ 2 (x/2)^{deg+1} / (deg+1)!);
// for x < 1e-3 the Taylor polynomial, which is then as accurate.  Returned in the nested form
// the stencil evaluates,
//     p(z) v = a_0 (v + r_1 z (v + r_2 z (v + ... + r_deg z v))),   r_k = a_k / a_{k-1},
// with a0 = a_0 and ratio[k] = r_k (k = 1..deg, ratio[0] unused).  Returns the largest
// |p(z) - e^z| over 4001 evenly spaced points of [-x, x] (in long double), or a negative value
// when deg is outside 1..kMaxPolyDeg or some a_k is not positive (the nested form needs a_k > 0).
constexpr int kMaxPolyDeg = 10;
double exp_poly_ratios(double x, int deg, double* a0, double* ratio);

}  // namespace hub
