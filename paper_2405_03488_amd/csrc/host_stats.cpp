// Online convergence detection (Sec. 4.1): exact sums, predicted error, windows.
//
// The NS-online algorithm keeps sum and squaredSum of the sampled counts and,
// at the end of every window, computes mu = sum/n, var = squaredSum/n - mu^2,
// sigma = sqrt(var/n) and the predicted error z*sigma/mu (error equation) with
// z = Phi^-1(1 - delta/2); it stops once that is at most eps.  Here the sums
// are exact integers, and the predicted error is evaluated as
//     eps_hat = z * sqrt(D / n) / S1,   D = n*S2 - S1^2   (exact, >= 0),
// which equals the paper's expression algebraically without the cancellation
// of var = S2/n - mu^2.  D, S1 are rounded to double once (nearest, ties to
// even); eps_hat = +inf while S1 = 0.
#include <cmath>

#include "sgpm_internal.h"

namespace sgpm {

void big_add_digits(Big& a, const unsigned long long* digits, int nd) {
    // digits[i] weighs 2^(32 i) and may exceed 32 bits
    unsigned __int128 carry = 0;
    for (size_t i = 0; i < a.d.size(); i++) {
        unsigned __int128 t = carry + a.d[i];
        if ((int)i < nd) t += digits[i];
        a.d[i] = (uint32_t)t;
        carry = t >> 32;
    }
}

bool big_is_zero(const Big& a) {
    for (uint32_t x : a.d)
        if (x) return false;
    return true;
}

static int bit_length(const Big& a) {
    for (int i = (int)a.d.size() - 1; i >= 0; i--)
        if (a.d[(size_t)i]) return 32 * i + 32 - __builtin_clz(a.d[(size_t)i]);
    return 0;
}

static uint64_t bits_at(const Big& a, int lo) {  // 64 bits starting at bit lo (lo >= 0)
    uint64_t r = 0;
    for (int b = 0; b < 64; b++) {
        int i = lo + b;
        if (i / 32 < (int)a.d.size() && (a.d[(size_t)(i / 32)] >> (i % 32) & 1)) r |= 1ull << b;
    }
    return r;
}

double big_to_double(const Big& a) {
    int L = bit_length(a);
    if (L == 0) return 0.0;
    if (L <= 64) return (double)bits_at(a, 0);  // the conversion rounds to nearest even
    int shift = L - 64;
    uint64_t top = bits_at(a, shift);
    bool sticky = false;
    for (int i = 0; i < shift && !sticky; i++) sticky = a.d[(size_t)(i / 32)] >> (i % 32) & 1;
    uint64_t keep = top >> 11, rem = top & 0x7FF;
    if (rem > 0x400 || (rem == 0x400 && (sticky || (keep & 1)))) keep++;
    return std::ldexp((double)keep, shift + 11);
}

static Big big_mul(const Big& a, const Big& b) {
    Big r(a.d.size());
    for (size_t i = 0; i < a.d.size(); i++) {
        if (!a.d[i]) continue;
        unsigned __int128 carry = 0;
        for (size_t j = 0; i + j < r.d.size(); j++) {
            unsigned __int128 t = (unsigned __int128)a.d[i] * b.d[j] + r.d[i + j] + carry;
            r.d[i + j] = (uint32_t)t;
            carry = t >> 32;
        }
    }
    return r;
}

static bool big_sub(Big& a, const Big& b) {  // a -= b, false on underflow
    int64_t borrow = 0;
    for (size_t i = 0; i < a.d.size(); i++) {
        int64_t t = (int64_t)a.d[i] - (int64_t)b.d[i] - borrow;
        borrow = t < 0 ? 1 : 0;
        a.d[i] = (uint32_t)(t & 0xFFFFFFFFll);
    }
    return borrow == 0;
}

// Phi^-1(p), 0.5 < p < 1: Newton's method on Phi(x) = erfc(-x/sqrt2)/2 in
// extended precision, then rounded to double.
double normal_quantile(double p) {
    if (!(p > 0.5 && p < 1.0)) return NAN;
    long double x = 1.0L, P = p;
    const long double rs2 = 0.70710678118654752440084436210484903L;
    const long double rs2pi = 0.39894228040143267793994605993438187L;
    for (int it = 0; it < 200; it++) {
        long double f = 0.5L * erfcl(-x * rs2) - P;
        long double dens = rs2pi * expl(-0.5L * x * x);
        long double nx = x - f / dens;
        if (nx == x) break;
        x = nx;
    }
    return (double)x;
}

// Regularised incomplete beta I_x(a, b) in extended precision: the continued
// fraction of Abramowitz and Stegun 26.5.8, evaluated by the modified Lentz
// method, on the side of the symmetry I_x(a, b) = 1 - I_{1-x}(b, a) where it
// converges quickly (x < (a + 1) / (a + b + 2)).
static long double incomplete_beta(long double x, long double a, long double b) {
    if (x <= 0.0L) return 0.0L;
    if (x >= 1.0L) return 1.0L;
    if (x > (a + 1.0L) / (a + b + 2.0L)) return 1.0L - incomplete_beta(1.0L - x, b, a);
    const long double tiny = 1e-4000L;
    const long double lead =
        expl(a * logl(x) + b * log1pl(-x) + lgammal(a + b) - lgammal(a) - lgammal(b)) / a;
    long double f = 1.0L, C = 1.0L, D = 0.0L;
    for (int i = 1; i < 100000; i++) {
        const int m = i / 2;
        long double d;
        if (i % 2) d = -(a + m) * (a + b + m) * x / ((a + 2 * m) * (a + 2 * m + 1));
        else d = m * (b - m) * x / ((a + 2 * m - 1) * (a + 2 * m));
        D = 1.0L + d * D;
        if (fabsl(D) < tiny) D = tiny;
        C = 1.0L + d / C;
        if (fabsl(C) < tiny) C = tiny;
        D = 1.0L / D;
        const long double step = C * D;
        f *= step;
        if (fabsl(step - 1.0L) < 1e-21L) break;
    }
    // the fraction's leading term 1 / (1 + d1 / (1 + ...)) with f = 1 + d1/(1 + ...)
    return lead / f;
}

// Two-sided Student t quantile: t with P(|T| <= t) = conf for nu degrees of
// freedom, where P(|T| <= t) = 1 - I_{nu / (nu + t^2)}(nu / 2, 1 / 2).  Newton's
// method from the normal quantile, with the density 2 f(t) as the derivative,
// kept inside a bracket that halves whenever a Newton step leaves it.
double student_t_quantile(double conf, int nu) {
    if (!(conf > 0.0 && conf < 1.0) || nu < 1) return NAN;
    const long double v = nu, C = conf;
    auto central = [&](long double t) { return 1.0L - incomplete_beta(v / (v + t * t), v / 2.0L, 0.5L); };
    const long double logc = lgammal((v + 1.0L) / 2.0L) - lgammal(v / 2.0L) - 0.5L * logl(v * 3.14159265358979323846L);
    auto dens2 = [&](long double t) { return 2.0L * expl(logc - (v + 1.0L) / 2.0L * log1pl(t * t / v)); };
    long double lo = 0.0L, hi = 1.0L;
    while (central(hi) < C) hi *= 2.0L;
    long double t = normal_quantile(0.5 + conf / 2.0);
    if (!(t > lo && t < hi)) t = 0.5L * (lo + hi);
    for (int it = 0; it < 400; it++) {
        const long double f = central(t) - C;
        if (f < 0) lo = t; else hi = t;
        long double nt = t - f / dens2(t);
        if (!(nt > lo && nt < hi)) nt = 0.5L * (lo + hi);
        if (nt == t || hi - lo <= 0.0L) break;
        t = nt;
    }
    return (double)t;
}

// Predicted relative error of the mean of n i.i.d. values with the unbiased
// sample variance: t * sqrt(D / (n - 1)) / S1, D = n S2 - S1^2 (exact); +inf
// while n < 2 or S1 = 0.  The GS path's repeated sparsifications use it with
// the Student t quantile of n - 1 degrees of freedom.
double predicted_error_t(double t, uint64_t n, const Big& S1, const Big& S2) {
    if (n < 2 || big_is_zero(S1)) return INFINITY;
    Big N(S2.d.size());
    N.d[0] = (uint32_t)n;
    N.d[1] = (uint32_t)(n >> 32);
    Big D = big_mul(N, S2);
    Big S1sq = big_mul(S1, S1);
    if (!big_sub(D, S1sq)) return NAN;
    double dD = big_to_double(D), dn1 = (double)(n - 1), dS1 = big_to_double(S1);
    double q = dD / dn1;
    double r = std::sqrt(q);
    double u = t * r;
    return u / dS1;
}

double predicted_error(double z, uint64_t n, const Big& S1, const Big& S2) {
    if (n == 0 || big_is_zero(S1)) return INFINITY;
    Big N(S2.d.size());
    N.d[0] = (uint32_t)n;
    N.d[1] = (uint32_t)(n >> 32);
    Big D = big_mul(N, S2);
    Big S1sq = big_mul(S1, S1);
    if (!big_sub(D, S1sq)) return NAN;
    double dD = big_to_double(D), dn = (double)n, dS1 = big_to_double(S1);
    double q = dD / dn;
    double r = std::sqrt(q);
    double t = z * r;
    return t / dS1;
}

uint64_t next_window_end(uint64_t n_t, const sgpm_options& o) {
    auto up = [&](uint64_t x) { return o.quantum ? (x + o.quantum - 1) / o.quantum * o.quantum : x; };
    uint64_t nx;
    if (n_t == 0) {
        nx = up(o.n_min);
    } else {
        uint64_t inc = (uint64_t)std::ceil(o.window_growth * (double)n_t);
        if (inc < o.w_min) inc = o.w_min;
        nx = up(n_t + inc);
    }
    if (o.max_samples && nx > o.max_samples) nx = o.max_samples;
    return nx;
}

}  // namespace sgpm
