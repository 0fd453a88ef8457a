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
