// Wigner d^l_{ab}(pi/2) chains for the contraction kernels and the plan.
//
// Two three-term recursions at beta = pi/2 (identities of the Wigner
// functions; the paper's own recursion choice is Risbo's, Section 2.2):
//
//  (in l, fixed a, b)   l sqrt(((l+1)^2-a^2)((l+1)^2-b^2)) d^{l+1}
//                         = -(2l+1) a b d^l - (l+1) sqrt((l^2-a^2)(l^2-b^2)) d^{l-1}
//  (in a, fixed l, b)   sqrt((l+a)(l-a+1)) d_{a-1,b} + sqrt((l-a)(l+a+1)) d_{a+1,b}
//                         = 2 b d_{a,b}
//
// Both start on the edge max(|a|, |b|) = l0 of the (a, b) square, where the
// closed forms are
//   d^l_{l,b} = (-1)^{l-b} E(l,|b|),   d^l_{-l,b} = E(l,|b|),
//   d^l_{a,l} = E(l,|a|),              d^l_{a,-l} = (-1)^{l+a} E(l,|a|),
// with E(l,k) = 2^-l sqrt(C(2l, l+k)) (EdgeTable, extended exponent).
#pragma once

#include "sht_internal.h"

namespace sht {

// Seed of a chain as (scaled value, scale level): value = v * 2^(-512 k).
struct Seed {
    double v;
    int k;
};

__device__ inline Seed edge_value(const EdgeTable &E, int l, int kk, double sign) {
    const long long idx = (long long)l * (l + 1) / 2 + kk;
    const double mant = E.mant[idx];
    const int ex = E.expo[idx];           // <= 0
    const int k = (-ex) / 512;
    Seed s;
    s.v = sign * ldexp(mant, ex + 512 * k);
    s.k = k;
    return s;
}

// d^{l0}_{a,b}(pi/2) with l0 = max(|a|, |b|).
__device__ inline Seed edge_seed(const EdgeTable &E, int a, int b) {
    const int aa = a < 0 ? -a : a, bb = b < 0 ? -b : b;
    if (aa >= bb) {
        const int l = aa;
        if (a >= 0) return edge_value(E, l, bb, sgn_pow((long long)l - b));
        return edge_value(E, l, bb, 1.0);
    }
    const int l = bb;
    if (b >= 0) return edge_value(E, l, aa, 1.0);
    return edge_value(E, l, aa, sgn_pow((long long)l + a));
}

__device__ inline double emit_scale(int k) { return k == 0 ? 1.0 : (k == 1 ? kSmall : 0.0); }

// One chain carried through a recursion: current value d, previous value dp
// (both scaled by 2^(512 k)), and the factor that unscales an emitted value.
struct Chain {
    double d, dp, es;
    int k;

    __device__ inline void zero() { d = 0.0; dp = 0.0; es = 1.0; k = 0; }
    __device__ inline void inject(Seed s) { d = s.v; dp = 0.0; k = s.k; es = emit_scale(s.k); }
    // Accept a new value, keeping values below 2^512 in scaled form.
    __device__ inline void push(double dn) {
        dp = d;
        d = dn;
        if (k > 1 && fabs(d) > kBig) {
            d *= kSmall;
            dp *= kSmall;
            --k;
            es = emit_scale(k);
        }
    }
    __device__ inline double value() const { return d * es; }
};

// l-recursion factor for one index a at level l (l >= 1):
//   am = a / sqrt((l+1)^2 - a^2) * (2l+1)/l,  bm = sqrt(l^2 - a^2)/sqrt((l+1)^2 - a^2) * (l+1)/l
// so that d^{l+1}_{ab} = -(am(a) am'(b) d^l + bm(a) bm'(b) d^{l-1}) where the
// primed factors omit the l-dependent constants.  Out-of-range indices give
// finite values (their chains are still zero).
__device__ inline void lrec_factor_full(int l, int a, double &am, double &bm) {
    if (l == 0) { am = 0.0; bm = 0.0; return; }
    const double X = (double)(l + 1) * (l + 1) - (double)a * a;
    const double Y = (double)l * l - (double)a * a;
    const double r = rsqrt(X > 1.0 ? X : 1.0);
    am = (double)a * r * ((2.0 * l + 1.0) / l);
    bm = sqrt(Y > 0.0 ? Y : 0.0) * r * ((l + 1.0) / l);
}

}  // namespace sht
