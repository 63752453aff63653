// Driver for the address/undefined-behaviour sanitizer run of the host core
// (host_core.cpp, poly.cpp): exercises every host-only entry point of the C
// ABI and the Givens least squares on seeded random inputs, including the
// error paths, and checks the structural properties of each result. Built and
// run by tests/test_host_sanitizers.py with g++ (no GPU code involved).
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "../include/ppgmres.h"
#include "../paper_1911_07065_amd/csrc/host_core.h"

static int g_fail = 0;
#define CHECK(c)                                                               \
    do {                                                                       \
        if (!(c)) {                                                            \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
            ++g_fail;                                                          \
        }                                                                      \
    } while (0)

// Random roots: reals and exact conjugate pairs, with repeated values and
// integer ties so the ordering meets equal scores.
static void random_roots(std::mt19937_64 &g, int d, std::vector<double> &re, std::vector<double> &im) {
    std::uniform_real_distribution<double> u(-3.0, 12.0), v(0.05, 4.0);
    std::uniform_int_distribution<int> pick(0, 5);
    re.clear();
    im.clear();
    while ((int)re.size() < d) {
        const int k = pick(g);
        if (k == 0 && (int)re.size() + 2 <= d) {
            const double a = u(g), b = v(g);
            re.push_back(a), im.push_back(b);
            re.push_back(a), im.push_back(-b);
        } else if (k == 1 && !re.empty()) {
            re.push_back(re[0]), im.push_back(0.0);  // a duplicate of the first real part
            if (im.back() != 0.0) im.back() = 0.0;
        } else if (k == 2) {
            re.push_back((double)(1 + (int)(g() % 6))), im.push_back(0.0);  // integer ties
        } else {
            double a = u(g);
            if (a == 0.0) a = 1.0;
            re.push_back(a), im.push_back(0.0);
        }
    }
    for (int i = 0; i < d; ++i)
        if (re[i] == 0.0 && im[i] == 0.0) re[i] = 0.5;
}

static void roots_cases(std::mt19937_64 &g) {
    for (int t = 0; t < 300; ++t) {
        const int d = 1 + (int)(g() % 64);
        std::vector<double> re, im;
        random_roots(g, d, re, im);
        std::vector<int> perm(d, -1);
        CHECK(pp_leja_order(d, re.data(), im.data(), perm.data()) == PP_OK);
        std::vector<int> seen(d, 0);
        for (int i = 0; i < d; ++i) {
            CHECK(perm[i] >= 0 && perm[i] < d);
            if (perm[i] >= 0 && perm[i] < d) seen[perm[i]]++;
        }
        for (int i = 0; i < d; ++i) CHECK(seen[i] == 1);
        std::vector<double> ore(d), oim(d);
        for (int i = 0; i < d; ++i) ore[i] = re[perm[i]], oim[i] = im[perm[i]];
        for (int add = 0; add <= 1; ++add) {
            const int cap = d * 23;
            std::vector<double> fr(cap), fi(cap), pm(d);
            std::vector<int> na(d), pe(d);
            int d_eff = -1;
            CHECK(pp_add_roots(d, ore.data(), oim.data(), add, cap, fr.data(), fi.data(), &d_eff, na.data(),
                               pm.data(), pe.data()) == PP_OK);
            int extra = 0;
            for (int i = 0; i < d; ++i) extra += na[i];
            CHECK(d_eff >= d && d_eff <= cap);
            if (!add) CHECK(d_eff == d);
            // a too small output list is an error, not an overrun
            if (d_eff > 1) CHECK(pp_add_roots(d, ore.data(), oim.data(), add, d_eff - 1, fr.data(), fi.data(),
                                              &d_eff, na.data(), pm.data(), pe.data()) != PP_OK);
        }
        for (int flags = 0; flags <= 3; ++flags) {
            pp_poly p = nullptr;
            const double *r = flags & PP_ROOTS_KEEP_ORDER ? ore.data() : re.data();
            const double *s = flags & PP_ROOTS_KEEP_ORDER ? oim.data() : im.data();
            if (pp_poly_from_roots(d, r, s, flags, &p) != PP_OK) {
                CHECK(false);
                continue;
            }
            for (int which = 0; which <= 3; ++which) {
                int len = -1, dorig = -1, nadd = -1;
                const pp_status st = pp_poly_roots(p, which, 0, nullptr, nullptr, &len, &dorig, &nadd);
                if (which == PP_ROOTS_INNER) {
                    CHECK(st != PP_OK);  // not a composite polynomial
                    continue;
                }
                CHECK(st == PP_OK && len >= 1);
                std::vector<double> a(len), b(len);
                CHECK(pp_poly_roots(p, which, len, a.data(), b.data(), &len, &dorig, &nadd) == PP_OK);
                if (len > 1) CHECK(pp_poly_roots(p, which, len - 1, a.data(), b.data(), &len, nullptr, nullptr) != PP_OK);
            }
            pp_poly_destroy(p);
        }
    }
    // unpaired complex root and bad arguments
    double re1[2] = {1.0, 2.0}, im1[2] = {0.5, 0.0};
    int perm[2];
    CHECK(pp_leja_order(2, re1, im1, perm) != PP_OK);
    CHECK(pp_leja_order(0, re1, im1, perm) != PP_OK);
    pp_poly p = nullptr;
    CHECK(pp_poly_from_roots(2, re1, im1, 0, &p) != PP_OK);
    CHECK(pp_poly_from_roots(2, re1, im1, 0, nullptr) != PP_OK);
}

static void hessenberg_cases(std::mt19937_64 &g) {
    std::normal_distribution<double> nd(0.0, 1.0);
    for (int t = 0; t < 150; ++t) {
        const int k = 1 + (int)(g() % 80);
        std::vector<double> hb((size_t)(k + 1) * k, 0.0);
        for (int j = 0; j < k; ++j)
            for (int i = 0; i <= j + 1 && i <= k; ++i) hb[(size_t)j * (k + 1) + i] = nd(g) + (i == j ? 3.0 : 0.0);
        std::vector<double> re(k), im(k);
        const pp_status st = pp_harmonic_ritz(k, hb.data(), (int)(t % 5 == 0), re.data(), im.data());
        CHECK(st == PP_OK || st == PP_ESINGULAR);
        if (st == PP_OK)
            for (int i = 0; i < k; ++i) CHECK(std::isfinite(re[i]) && std::isfinite(im[i]));
        CHECK(pp_hessenberg_eig(k, hb.data(), k + 1, re.data(), im.data()) == PP_OK);
        // eigenvalue sum equals the trace of the leading k x k block
        double tr = 0.0, sr = 0.0, si = 0.0;
        for (int i = 0; i < k; ++i) tr += hb[(size_t)i * (k + 1) + i], sr += re[i], si += im[i];
        CHECK(std::fabs(tr - sr) <= 1e-8 * (1.0 + std::fabs(tr)) * k);
        CHECK(std::fabs(si) <= 1e-8 * k);
    }
    // a singular leading block (zero column) is reported, not divided through
    std::vector<double> z(3 * 2, 0.0);
    double re[2], im[2];
    CHECK(pp_harmonic_ritz(2, z.data(), 0, re, im) == PP_ESINGULAR);
    CHECK(pp_harmonic_ritz(0, z.data(), 0, re, im) != PP_OK);
}

static void givens_cases(std::mt19937_64 &g) {
    std::normal_distribution<double> nd(0.0, 1.0);
    for (int t = 0; t < 100; ++t) {
        const int m = 1 + (int)(g() % 60);
        ppg::GivensLS ls;
        const double beta = 1.0 + std::fabs(nd(g));
        ls.reset(m, beta);
        std::vector<double> col(m + 1);
        double last = beta;
        for (int j = 0; j < m; ++j) {
            for (int i = 0; i <= j + 1; ++i) col[i] = nd(g) + (i == j ? 4.0 : 0.0);
            const double r = ls.add_column(col.data());
            CHECK(std::isfinite(r) && r <= last * (1.0 + 1e-12));  // the residual never grows
            last = r;
        }
        std::vector<double> z(m);
        ls.solve(z.data());
        for (int i = 0; i < m; ++i) CHECK(std::isfinite(z[i]));
    }
}

int main() {
    std::mt19937_64 g(20191115);
    roots_cases(g);
    hessenberg_cases(g);
    givens_cases(g);
    if (g_fail) {
        std::fprintf(stderr, "%d checks failed\n", g_fail);
        return 1;
    }
    std::printf("host core sanitizer run: ok\n");
    return 0;
}
