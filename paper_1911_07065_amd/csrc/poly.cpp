// Chain programs: the sequence of fused launches that evaluates phi(A)v,
// pi(A)v (Algorithm 1) or p(A)v (Algorithm 3) for an ordered root list.
#include "poly.h"

#include <atomic>

namespace ppg {

unsigned long long next_poly_id() {
    static std::atomic<unsigned long long> counter{0};
    return ++counter;
}

namespace {

Step make(int spmv, int in, int aux, int out, int acc, int acc_init, int fin, double a0, double a1, double a2,
          double b0, double b1) {
    Step s;
    s.spmv = spmv;
    s.in = in;
    s.aux = aux;
    s.out = out;
    s.acc = acc;
    s.acc_init = acc_init;
    s.fin = fin;
    s.a0 = a0;
    s.a1 = a1;
    s.a2 = a2;
    s.b0 = b0;
    s.b1 = b1;
    return s;
}

}  // namespace

// Algorithm 1: pi <- pi - (1/theta) A pi for a real root; for a pair
// a +/- bi: t = A pi, pi <- pi + (A t - 2 a t)/(a^2 + b^2) (eq. 2.2);
// finally phi = v - pi (fused into the last launch).
std::vector<Step> program_phi(const std::vector<Unit> &units, bool want_pi) {
    std::vector<Step> prog;
    int cur = B_IN;
    int toggle = 0;
    const int L = (int)units.size();
    for (int idx = 0; idx < L; ++idx) {
        const Unit &u = units[idx];
        const bool last = idx == L - 1;
        const int out = last ? B_OUT : ((toggle++ & 1) ? B_P1 : B_P0);
        const int fin = (last && !want_pi) ? 1 : 0;
        if (u.kind == UNIT_REAL) {
            const double c = 1.0 / u.re;
            prog.push_back(make(1, cur, B_NONE, out, B_NONE, 0, fin, -c, 1.0, 0.0, 0.0, 0.0));
        } else {
            const double s = 1.0 / (u.re * u.re + u.im * u.im);
            prog.push_back(make(1, cur, B_NONE, B_T, B_NONE, 0, 0, 1.0, 0.0, 0.0, 0.0, 0.0));
            prog.push_back(make(1, B_T, cur, out, B_NONE, 0, fin, s, -2.0 * u.re * s, 1.0, 0.0, 0.0));
        }
        cur = out;
    }
    return prog;
}

// Algorithm 3 (eq. 3.1): p accumulates (1/theta_k) prod for real roots and
// prod (2a - A)/(a^2+b^2) for pairs, while prod advances by the factor
// (1 - A/theta_k) or its folded pair form. The last unit only contributes
// to p; when it is real its contribution c*prod is added by the launch
// that produced prod, so p(A)v costs d_eff - 1 sparse products.
std::vector<Step> program_p(const std::vector<Unit> &units) {
    std::vector<Step> prog;
    const int L = (int)units.size();
    if (L == 1 && units[0].kind == UNIT_REAL) {
        prog.push_back(make(0, B_IN, B_NONE, B_NONE, B_OUT, 1, 0, 0.0, 0.0, 0.0, 1.0 / units[0].re, 0.0));
        return prog;
    }
    int cur = B_IN;
    int toggle = 0;
    int first = 1;
    for (int idx = 0; idx < L; ++idx) {
        const Unit &u = units[idx];
        const bool last = idx == L - 1;
        const bool next_is_last_real = (idx + 1 == L - 1) && units[L - 1].kind == UNIT_REAL;
        const double c_next = next_is_last_real ? 1.0 / units[L - 1].re : 0.0;
        if (u.kind == UNIT_REAL) {
            if (last) break;  // folded into the previous launch
            const double c = 1.0 / u.re;
            const int out = next_is_last_real ? B_NONE : ((toggle++ & 1) ? B_P1 : B_P0);
            prog.push_back(make(1, cur, B_NONE, out, B_OUT, first, 0, -c, 1.0, 0.0, c, c_next));
            cur = out;
        } else {
            const double s = 1.0 / (u.re * u.re + u.im * u.im);
            prog.push_back(make(1, cur, B_NONE, last ? B_NONE : B_T, B_OUT, first, 0, -1.0, 2.0 * u.re, 0.0, 0.0,
                                s));
            if (!last) {
                first = 0;
                const int out = next_is_last_real ? B_NONE : ((toggle++ & 1) ? B_P1 : B_P0);
                prog.push_back(make(1, B_T, cur, out, B_OUT, 0, 0, -s, 0.0, 1.0, 0.0, c_next));
                cur = out;
            }
        }
        first = 0;
    }
    return prog;
}

}  // namespace ppg
