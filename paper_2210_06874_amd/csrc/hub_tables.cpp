// Host-side FP64 tables: mixed-radix plan, DFT roots of unity and the momentum-space
// hopping exponential E(k) = exp(delta*kappa*K(k)) of the honeycomb torus.
//
// In momentum space (Bloch theorem on the L x L torus) the hopping matrix of the
// honeycomb lattice (paper Sec. 1, fig. "honeycomb_lattice") is the 2 x 2 block
// K(k) = [[0, f(k)], [conj f(k), 0]], f(k) = 1 + e^{-i k1} + e^{-i k2}, whose
// eigenvalues +-|f(k)| are the two free bands of Sec. 1.  Because K(k)^2 = |f|^2,
//     exp(dk K(k)) = cosh(dk|f|) 1 + sinh(dk|f|)/|f| K(k).
// A chemical potential mu multiplies every time hop by e^{delta mu} (Sec. 1 Hamiltonian:
// mu couples to the charge; Sec. 3 weight det(M[phi,mu] M[phi,-mu]^dag)).
#include <cmath>

#include "hub_tables.hpp"

namespace hub {

static const int kRadices[] = {4, 2, 3, 5, 7, 11, 13, 17};

bool make_plan(int L, FftPlan* plan) {
    if (L < 1 || L > 1024) return false;
    plan->L = L;
    plan->nst = 0;
    int rest = L;
    // Extract factors of 4 first, then the other supported primes.
    for (int r : kRadices) {
        while (rest % r == 0) {
            if (plan->nst >= kMaxStages) return false;
            plan->radix[plan->nst++] = r;
            rest /= r;
        }
    }
    if (rest != 1) return false;
    int len = L;
    for (int q = 0; q < plan->nst; ++q) {
        plan->len[q] = len;
        len /= plan->radix[q];
    }
    return true;
}

int digit_reversed_position(const FftPlan& plan, int k) {
    // k = k_0 + r_0 k_1 + r_0 r_1 k_2 + ...; after stage q the digit k_q sits at
    // stride len[q] / radix[q] inside its block.
    int pos = 0;
    for (int q = 0; q < plan.nst; ++q) {
        const int r = plan.radix[q];
        pos += (k % r) * (plan.len[q] / r);
        k /= r;
    }
    return pos;
}

void build_tables(const FftPlan& plan, double dk, double dmu, std::vector<double>& roots,
                  std::vector<double>& etab) {
    const int L = plan.L;
    const double two_pi = 6.283185307179586476925286766559;
    roots.assign(2 * (size_t)L, 0.0);
    for (int m = 0; m < L; ++m) {
        const double a = two_pi * (double)m / (double)L;   // m < L: exact integer numerator
        roots[2 * m] = std::cos(a);
        roots[2 * m + 1] = -std::sin(a);
    }
    std::vector<int> inv_pos(L);
    for (int k = 0; k < L; ++k) inv_pos[digit_reversed_position(plan, k)] = k;
    etab.assign(4 * (size_t)L * L, 0.0);
    const double norm = std::exp(dmu) / ((double)L * (double)L);
    for (int p1 = 0; p1 < L; ++p1) {
        const int k1 = inv_pos[p1];
        for (int p2 = 0; p2 < L; ++p2) {
            const int k2 = inv_pos[p2];
            const double fr = 1.0 + roots[2 * k1] + roots[2 * k2];
            const double fi = roots[2 * k1 + 1] + roots[2 * k2 + 1];
            const double af = std::hypot(fr, fi);
            const double x = dk * af;
            const double c = std::cosh(x);
            double s;
            if (std::fabs(x) < 1e-4) {
                // sinh(x)/x series (even in x, so either sign of dk); |f| may vanish exactly
                // at the Dirac momenta
                const double x2 = x * x;
                s = dk * (1.0 + x2 / 6.0 * (1.0 + x2 / 20.0));
            } else {
                s = std::sinh(x) / af;
            }
            double* e = &etab[4 * ((size_t)p1 * L + p2)];
            e[0] = c * norm;
            e[1] = s * fr * norm;
            e[2] = s * fi * norm;
            e[3] = 0.0;
        }
    }
}

double exp_poly_ratios(double x, int deg, double* a0, double* ratio) {
    if (deg < 1 || deg > kMaxPolyDeg || !(x >= 0.0) || !std::isfinite(x)) return -1.0;
    const int n = deg + 1;
    long double a[kMaxPolyDeg + 1] = {};
    const long double xl = x;
    if (x < 1e-3) {
        a[0] = 1.0L;
        for (int k = 1; k < n; ++k) a[k] = a[k - 1] / k;
    } else {
        // Chebyshev series of e^{x t} on [-1, 1]: e^{x t} = I_0(x) + 2 sum_{j>=1} I_j(x) T_j(t),
        // I_j(x) = sum_m (x/2)^{2m+j} / (m! (m+j)!) (every term positive), truncated at deg
        long double cj[kMaxPolyDeg + 1];
        for (int j = 0; j < n; ++j) {
            long double term = 1.0L;
            for (int i = 1; i <= j; ++i) term *= (xl / 2.0L) / i;     // (x/2)^j / j!
            long double s = 0.0L;
            for (int m = 0; m < 40 && term > 0.0L; ++m) {
                s += term;
                term *= (xl / 2.0L) * (xl / 2.0L) / ((m + 1.0L) * (m + 1.0L + j));
            }
            cj[j] = j == 0 ? s : 2.0L * s;
        }
        // monomial coefficients of T_j: T_0 = 1, T_1 = t, T_{j+1} = 2 t T_j - T_{j-1}
        long double T[kMaxPolyDeg + 1][kMaxPolyDeg + 1] = {};
        T[0][0] = 1.0L;
        if (n > 1) T[1][1] = 1.0L;
        for (int j = 1; j + 1 < n; ++j)
            for (int k = 0; k < n; ++k)
                T[j + 1][k] = (k > 0 ? 2.0L * T[j][k - 1] : 0.0L) - T[j - 1][k];
        long double xp = 1.0L;
        for (int k = 0; k < n; ++k) {                                 // a_k = b_k / x^k
            long double bk = 0.0L;
            for (int j = k; j < n; ++j) bk += cj[j] * T[j][k];
            a[k] = bk / xp;
            xp *= xl;
        }
    }
    for (int k = 0; k < n; ++k)
        if (!(a[k] > 0.0L)) return -1.0;
    *a0 = (double)a[0];
    ratio[0] = 0.0;
    for (int k = 1; k < n; ++k) ratio[k] = (double)(a[k] / a[k - 1]);
    long double err = 0.0L;
    for (int i = 0; i <= 4000; ++i) {
        const long double z = xl * (-1.0L + i / 2000.0L);
        long double p = a[deg];
        for (int k = deg - 1; k >= 0; --k) p = a[k] + z * p;
        const long double d = p - std::exp(z);
        err = std::fmax(err, d < 0 ? -d : d);
    }
    return (double)err;
}

}  // namespace hub
