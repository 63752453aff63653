// Host-side building blocks: Hessenberg eigenvalues, harmonic Ritz values,
// modified Leja ordering, pof / added roots (Algorithm 2), Givens least
// squares. Compiled with -ffp-contract=off: no fused multiply-adds, so the
// integer results (orderings, counts, positions) are reproducible bit for
// bit in any IEEE binary64 implementation of the same rules.
#include "host_core.h"

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <new>
#include <utility>

#include "../../include/ppgmres.h"
#include "poly.h"

namespace ppg {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

// ---------------------------------------------------------------------------
// Francis double-shift QR on an upper Hessenberg matrix (eigenvalues only).
// Golub & Van Loan, Matrix Computations, section 7.5: implicit double shift
// with 3x3 Householder bulge chasing, deflation at negligible subdiagonals.
// ---------------------------------------------------------------------------

namespace {

struct Mat {
    int n;
    std::vector<double> a;  // column-major
    double &operator()(int i, int j) { return a[(size_t)i + (size_t)j * n]; }
    double operator()(int i, int j) const { return a[(size_t)i + (size_t)j * n]; }
};

// Eigenvalues of [[a, b], [c, d]]; a complex pair comes out as exact conjugates.
void eig2x2(double a, double b, double c, double d, double *re, double *im) {
    double p = 0.5 * (a - d);
    double bc = b * c;
    double q = p * p + bc;
    if (q >= 0.0) {
        double r = std::sqrt(q);
        double z = (p >= 0.0) ? p + r : p - r;
        re[0] = d + z;
        re[1] = (z != 0.0) ? d - bc / z : d;
        im[0] = 0.0;
        im[1] = 0.0;
    } else {
        double mid = d + p;
        double w = std::sqrt(-q);
        re[0] = mid;
        re[1] = mid;
        im[0] = w;
        im[1] = -w;
    }
}

// Householder vector for u (len 2 or 3): (I - beta v v^T) u = alpha e1.
double house(const double *u, int len, double *v) {
    double nrm2 = 0.0;
    for (int i = 0; i < len; ++i) nrm2 += u[i] * u[i];
    double nrm = std::sqrt(nrm2);
    for (int i = 0; i < len; ++i) v[i] = u[i];
    if (nrm == 0.0) return 0.0;
    double alpha = (u[0] >= 0.0) ? -nrm : nrm;
    v[0] = u[0] - alpha;
    double vv = 0.0;
    for (int i = 0; i < len; ++i) vv += v[i] * v[i];
    if (vv == 0.0) return 0.0;
    return 2.0 / vv;
}

void reflect_rows(Mat &H, int r0, int len, const double *v, double beta, int c0, int c1) {
    for (int c = c0; c <= c1; ++c) {
        double dot = 0.0;
        for (int i = 0; i < len; ++i) dot += v[i] * H(r0 + i, c);
        dot *= beta;
        for (int i = 0; i < len; ++i) H(r0 + i, c) -= dot * v[i];
    }
}

void reflect_cols(Mat &H, int c0, int len, const double *v, double beta, int r0, int r1) {
    for (int r = r0; r <= r1; ++r) {
        double dot = 0.0;
        for (int i = 0; i < len; ++i) dot += H(r, c0 + i) * v[i];
        dot *= beta;
        for (int i = 0; i < len; ++i) H(r, c0 + i) -= dot * v[i];
    }
}

}  // namespace

bool hessenberg_eig(int k, const double *h, int ld, double *re, double *im) {
    Mat H{k, std::vector<double>((size_t)k * k, 0.0)};
    double scale = 0.0;
    for (int j = 0; j < k; ++j)
        for (int i = 0; i <= std::min(j + 1, k - 1); ++i) {
            H(i, j) = h[(size_t)i + (size_t)j * ld];
            scale += std::fabs(H(i, j));
        }
    const double eps = DBL_EPSILON;
    int hi = k - 1;
    int iter = 0;
    long total = 0;
    const long max_total = 100L * std::max(k, 10);
    while (hi >= 0) {
        if (hi == 0) {
            re[0] = H(0, 0);
            im[0] = 0.0;
            break;
        }
        int lo = hi;
        while (lo > 0) {
            double s = std::fabs(H(lo - 1, lo - 1)) + std::fabs(H(lo, lo));
            if (s == 0.0) s = scale;
            if (std::fabs(H(lo, lo - 1)) <= eps * s) {
                H(lo, lo - 1) = 0.0;
                break;
            }
            --lo;
        }
        if (lo == hi) {
            re[hi] = H(hi, hi);
            im[hi] = 0.0;
            --hi;
            iter = 0;
            continue;
        }
        if (lo == hi - 1) {
            eig2x2(H(hi - 1, hi - 1), H(hi - 1, hi), H(hi, hi - 1), H(hi, hi), re + hi - 1, im + hi - 1);
            hi -= 2;
            iter = 0;
            continue;
        }
        if (++total > max_total) return false;
        ++iter;
        double s, t;
        if (iter % 11 == 10) {  // exceptional shift against cycling
            double w = std::fabs(H(hi, hi - 1)) + std::fabs(H(hi - 1, hi - 2));
            s = 1.5 * w;
            t = w * w;
        } else {
            s = H(hi - 1, hi - 1) + H(hi, hi);
            t = H(hi - 1, hi - 1) * H(hi, hi) - H(hi - 1, hi) * H(hi, hi - 1);
        }
        double u[3], v[3];
        u[0] = H(lo, lo) * H(lo, lo) + H(lo, lo + 1) * H(lo + 1, lo) - s * H(lo, lo) + t;
        u[1] = H(lo + 1, lo) * (H(lo, lo) + H(lo + 1, lo + 1) - s);
        u[2] = H(lo + 1, lo) * H(lo + 2, lo + 1);
        for (int kk = lo; kk <= hi - 2; ++kk) {
            double beta = house(u, 3, v);
            if (beta != 0.0) {
                reflect_rows(H, kk, 3, v, beta, std::max(lo, kk - 1), hi);
                reflect_cols(H, kk, 3, v, beta, lo, std::min(kk + 3, hi));
            }
            u[0] = H(kk + 1, kk);
            u[1] = H(kk + 2, kk);
            if (kk < hi - 2) u[2] = H(kk + 3, kk);
        }
        double beta = house(u, 2, v);
        if (beta != 0.0) {
            reflect_rows(H, hi - 1, 2, v, beta, hi - 2, hi);
            reflect_cols(H, hi - 1, 2, v, beta, lo, hi);
        }
        // clean the bulge remnants below the subdiagonal
        for (int j = lo; j <= hi; ++j)
            for (int i = j + 2; i <= hi; ++i) H(i, j) = 0.0;
    }
    return true;
}

// ---------------------------------------------------------------------------
// Harmonic Ritz values (Algorithm 4 step 1b)
// ---------------------------------------------------------------------------

int harmonic_ritz(int k, const double *hbar, bool breakdown, double *re, double *im) {
    const int ld = k + 1;
    std::vector<double> M((size_t)k * k);
    for (int j = 0; j < k; ++j)
        for (int i = 0; i < k; ++i) M[(size_t)i + (size_t)j * k] = hbar[(size_t)i + (size_t)j * ld];
    if (!breakdown) {
        // solve H^T f = e_k by Gaussian elimination with partial pivoting
        std::vector<double> T((size_t)k * k);
        for (int j = 0; j < k; ++j)
            for (int i = 0; i < k; ++i) T[(size_t)i + (size_t)j * k] = M[(size_t)j + (size_t)i * k];
        std::vector<double> f(k, 0.0);
        f[k - 1] = 1.0;
        auto Tt = [&](int i, int j) -> double & { return T[(size_t)i + (size_t)j * k]; };
        for (int c = 0; c < k; ++c) {
            int piv = c;
            for (int r = c + 1; r < k; ++r)
                if (std::fabs(Tt(r, c)) > std::fabs(Tt(piv, c))) piv = r;
            if (Tt(piv, c) == 0.0) return PP_ESINGULAR;
            if (piv != c) {
                for (int j = 0; j < k; ++j) std::swap(Tt(c, j), Tt(piv, j));
                std::swap(f[c], f[piv]);
            }
            for (int r = c + 1; r < k; ++r) {
                double l = Tt(r, c) / Tt(c, c);
                if (l == 0.0) continue;
                for (int j = c; j < k; ++j) Tt(r, j) -= l * Tt(c, j);
                f[r] -= l * f[c];
            }
        }
        for (int r = k - 1; r >= 0; --r) {
            double s = f[r];
            for (int j = r + 1; j < k; ++j) s -= Tt(r, j) * f[j];
            f[r] = s / Tt(r, r);
        }
        double h = hbar[(size_t)k + (size_t)(k - 1) * ld];
        for (int i = 0; i < k; ++i) {
            if (!std::isfinite(f[i])) return PP_ESINGULAR;
            M[(size_t)i + (size_t)(k - 1) * k] += h * h * f[i];
        }
    }
    if (!hessenberg_eig(k, M.data(), k, re, im)) {
        set_error("Hessenberg QR iteration did not converge");
        return PP_EINVAL;
    }
    for (int i = 0; i < k; ++i) {
        if (!std::isfinite(re[i]) || !std::isfinite(im[i]) || (re[i] == 0.0 && im[i] == 0.0))
            return PP_ESINGULAR;
    }
    return PP_OK;
}

// ---------------------------------------------------------------------------
// Exact mantissa/exponent products
// ---------------------------------------------------------------------------

static inline MantExp me_mul(MantExp a, double f) {
    int e2 = 0;
    double m2 = std::frexp(a.m * f, &e2);
    return MantExp{m2, a.e + e2};
}

// a > b for non-negative values
static inline bool me_greater(const MantExp &a, const MantExp &b) {
    if (a.m == 0.0) return false;
    if (b.m == 0.0) return true;
    if (a.e != b.e) return a.e > b.e;
    return a.m > b.m;
}

static inline double absdiff(double ar, double ai, double br, double bi) {
    double dr = ar - br;
    double di = ai - bi;
    return std::sqrt(dr * dr + di * di);
}

// ---------------------------------------------------------------------------
// Modified Leja ordering
// ---------------------------------------------------------------------------

namespace {
struct LUnit {
    int kind;
    double re, im;
    int ip, imn;
};
}  // namespace

bool leja_order(int d, const double *re, const double *im, int *perm) {
    std::map<std::pair<double, double>, std::vector<int>> minus_pool;
    for (int i = 0; i < d; ++i)
        if (im[i] < 0) minus_pool[{re[i], -im[i]}].push_back(i);
    std::map<std::pair<double, double>, size_t> taken;
    std::vector<LUnit> units;
    size_t n_minus = 0;
    for (auto &kv : minus_pool) n_minus += kv.second.size();
    size_t used = 0;
    for (int i = 0; i < d; ++i) {
        if (im[i] == 0.0) {
            units.push_back({UNIT_REAL, re[i], 0.0, i, -1});
        } else if (im[i] > 0.0) {
            auto key = std::make_pair(re[i], im[i]);
            auto it = minus_pool.find(key);
            size_t t = taken[key];
            if (it == minus_pool.end() || t >= it->second.size()) {
                set_error("complex root without its conjugate");
                return false;
            }
            units.push_back({UNIT_PAIR, re[i], im[i], i, it->second[t]});
            taken[key] = t + 1;
            ++used;
        } else if (!(im[i] < 0.0)) {
            set_error("non-finite root");
            return false;
        }
    }
    if (used != n_minus) {
        set_error("complex root without its conjugate");
        return false;
    }
    std::stable_sort(units.begin(), units.end(), [](const LUnit &a, const LUnit &b) {
        if (a.re != b.re) return a.re < b.re;
        return a.im < b.im;
    });
    const int nu = (int)units.size();
    std::vector<char> placed(nu, 0);
    std::vector<MantExp> score(nu, MantExp{0.5, 1});
    int best = -1;
    double best_mod = -1.0;
    for (int u = 0; u < nu; ++u) {
        double a = units[u].re, b = units[u].im;
        double mod = std::sqrt(a * a + b * b);
        if (mod > best_mod) {
            best = u;
            best_mod = mod;
        }
    }
    int out = 0;
    for (int step = 0; step < nu; ++step) {
        placed[best] = 1;
        const LUnit &pu = units[best];
        perm[out++] = pu.ip;
        if (pu.kind == UNIT_PAIR) perm[out++] = pu.imn;
        double rr[2] = {pu.re, pu.re};
        double ri[2] = {pu.im, -pu.im};
        int nr = pu.kind == UNIT_PAIR ? 2 : 1;
        for (int u = 0; u < nu; ++u) {
            if (placed[u]) continue;
            MantExp s = score[u];
            for (int q = 0; q < nr; ++q) s = me_mul(s, absdiff(units[u].re, units[u].im, rr[q], ri[q]));
            score[u] = s;
        }
        if (step == nu - 1) break;
        best = -1;
        for (int u = 0; u < nu; ++u) {
            if (placed[u]) continue;
            if (best < 0 || me_greater(score[u], score[best])) best = u;
        }
    }
    return true;
}

bool units_of(int d, const double *re, const double *im, std::vector<Unit> &units, std::vector<int> &pos) {
    units.clear();
    pos.clear();
    int i = 0;
    while (i < d) {
        if (im[i] == 0.0) {
            units.push_back({UNIT_REAL, re[i], 0.0});
            pos.push_back(i);
            i += 1;
        } else {
            if (i + 1 >= d || re[i + 1] != re[i] || im[i + 1] != -im[i] || im[i] < 0) {
                set_error("ordered roots must hold conjugate pairs as (a+bi, a-bi)");
                return false;
            }
            units.push_back({UNIT_PAIR, re[i], im[i]});
            pos.push_back(i);
            i += 2;
        }
    }
    return true;
}

std::vector<MantExp> pof_values(int d, const double *re, const double *im, const std::vector<Unit> &units,
                                const std::vector<int> &pos) {
    std::vector<MantExp> out;
    out.reserve(units.size());
    for (size_t u = 0; u < units.size(); ++u) {
        MantExp s{0.5, 1};
        const double a = units[u].re, b = units[u].im;
        for (int i = 0; i < d; ++i) {
            if (i == pos[u]) continue;
            double num = absdiff(re[i], im[i], a, b);
            double den = std::sqrt(re[i] * re[i] + im[i] * im[i]);
            s = me_mul(s, num / den);
        }
        out.push_back(s);
    }
    return out;
}

static const int kMaxThresholds = 22;  // 1e4 .. 1e298

int n_add_from_pof(const MantExp &pof) {
    int count = 0;
    for (int j = 0; j < kMaxThresholds; ++j) {
        char buf[32];
        std::snprintf(buf, sizeof(buf), "1e%d", 4 + 14 * j);
        int e = 0;
        double m = std::frexp(std::strtod(buf, nullptr), &e);
        MantExp t{m, e};
        if (!me_greater(t, pof))
            ++count;  // pof >= threshold
        else
            break;
    }
    return count;
}

std::vector<Unit> insert_copies(const std::vector<Unit> &units, const std::vector<int> &n_add) {
    // list of (unit id, is_copy)
    std::vector<std::pair<int, int>> R;
    R.reserve(units.size() * 2);
    for (int k = 0; k < (int)units.size(); ++k) R.push_back({k, 0});
    for (int k = 0; k < (int)units.size(); ++k) {
        const int c = n_add[k];
        if (c == 0) continue;
        long s = 0;
        for (; s < (long)R.size(); ++s)
            if (R[s].first == k && R[s].second == 0) break;
        const long L = (long)R.size();
        for (int j = c; j >= 1; --j) {
            long q = s + 1 + ((long)j * (L - s - 1)) / c;
            R.insert(R.begin() + q, {k, 1});
        }
    }
    std::vector<Unit> out;
    out.reserve(R.size());
    for (auto &e : R) out.push_back(units[e.first]);
    return out;
}

int plan_roots(int d, const double *re, const double *im, bool add, RootPlan &out) {
    std::vector<int> perm(d);
    if (!leja_order(d, re, im, perm.data())) return PP_EINVAL;
    out.leja_re.resize(d);
    out.leja_im.resize(d);
    for (int i = 0; i < d; ++i) {
        out.leja_re[i] = re[perm[i]];
        out.leja_im[i] = im[perm[i]];
    }
    std::vector<Unit> units;
    std::vector<int> pos;
    if (!units_of(d, out.leja_re.data(), out.leja_im.data(), units, pos)) return PP_EINVAL;
    out.pof = pof_values(d, out.leja_re.data(), out.leja_im.data(), units, pos);
    out.n_add.assign(units.size(), 0);
    if (add)
        for (size_t u = 0; u < units.size(); ++u) out.n_add[u] = n_add_from_pof(out.pof[u]);
    out.units = insert_copies(units, out.n_add);
    out.d = d;
    out.d_eff = 0;
    for (auto &u : out.units) out.d_eff += (u.kind == UNIT_PAIR) ? 2 : 1;
    out.n_added = out.d_eff - d;
    return PP_OK;
}

// ---------------------------------------------------------------------------
// Givens least squares
// ---------------------------------------------------------------------------

void GivensLS::reset(int m_, double beta) {
    m = m_;
    R.assign((size_t)(m + 1) * m, 0.0);
    c.assign(m, 0.0);
    s.assign(m, 0.0);
    g.assign(m + 1, 0.0);
    g[0] = beta;
    k = 0;
}

double GivensLS::add_column(const double *h) {
    const int j = k;
    const int ld = m + 1;
    double *col = &R[(size_t)j * ld];
    for (int i = 0; i <= j + 1; ++i) col[i] = h[i];
    for (int i = 0; i < j; ++i) {
        double t1 = c[i] * col[i] + s[i] * col[i + 1];
        double t2 = -s[i] * col[i] + c[i] * col[i + 1];
        col[i] = t1;
        col[i + 1] = t2;
    }
    double a = col[j], b = col[j + 1];
    double cj, sj;
    if (b == 0.0) {
        cj = 1.0;
        sj = 0.0;
    } else if (std::fabs(b) > std::fabs(a)) {
        double tau = a / b;
        sj = 1.0 / std::sqrt(1.0 + tau * tau);
        cj = sj * tau;
    } else {
        double tau = b / a;
        cj = 1.0 / std::sqrt(1.0 + tau * tau);
        sj = cj * tau;
    }
    c[j] = cj;
    s[j] = sj;
    col[j] = cj * a + sj * b;
    col[j + 1] = 0.0;
    g[j + 1] = -sj * g[j];
    g[j] = cj * g[j];
    k = j + 1;
    return std::fabs(g[j + 1]);
}

void GivensLS::solve(double *z) const {
    const int ld = m + 1;
    for (int i = k - 1; i >= 0; --i) {
        double t = g[i];
        for (int j = i + 1; j < k; ++j) t -= R[(size_t)i + (size_t)j * ld] * z[j];
        z[i] = t / R[(size_t)i + (size_t)i * ld];
    }
}

}  // namespace ppg

// ---------------------------------------------------------------------------
// C ABI: host-only entry points
// ---------------------------------------------------------------------------

using namespace ppg;

extern "C" {

const char *pp_last_error(void) { return g_last_error.c_str(); }

const char *pp_version(void) { return "ppgmres-mi355x 0.1 (gfx950)"; }

pp_status pp_hessenberg_eig(int k, const double *h, int ld, double *re, double *im) {
    if (k <= 0 || !h || !re || !im || ld < k) {
        set_error("pp_hessenberg_eig: bad argument");
        return PP_EINVAL;
    }
    if (!hessenberg_eig(k, h, ld, re, im)) {
        set_error("pp_hessenberg_eig: QR iteration did not converge");
        return PP_EINVAL;
    }
    return PP_OK;
}

pp_status pp_harmonic_ritz(int k, const double *hbar, int breakdown, double *re, double *im) {
    if (k <= 0 || !hbar || !re || !im) {
        set_error("pp_harmonic_ritz: bad argument");
        return PP_EINVAL;
    }
    int st = harmonic_ritz(k, hbar, breakdown != 0, re, im);
    if (st == PP_ESINGULAR) set_error("pp_harmonic_ritz: singular H_kk or zero root");
    return (pp_status)st;
}

pp_status pp_leja_order(int d, const double *re, const double *im, int *perm) {
    if (d <= 0 || !re || !im || !perm) {
        set_error("pp_leja_order: bad argument");
        return PP_EINVAL;
    }
    return leja_order(d, re, im, perm) ? PP_OK : PP_EINVAL;
}

pp_status pp_add_roots(int d, const double *re, const double *im, int add, int cap, double *re_out,
                       double *im_out, int *d_eff, int *n_add, double *pof_mant, int *pof_exp) {
    if (d <= 0 || !re || !im) {
        set_error("pp_add_roots: bad argument");
        return PP_EINVAL;
    }
    std::vector<Unit> units;
    std::vector<int> pos;
    if (!units_of(d, re, im, units, pos)) return PP_EINVAL;
    auto pof = pof_values(d, re, im, units, pos);
    std::vector<int> na(units.size(), 0);
    for (size_t u = 0; u < units.size(); ++u) {
        na[u] = add ? n_add_from_pof(pof[u]) : 0;
        int p = pos[u];
        int mem = units[u].kind == UNIT_PAIR ? 2 : 1;
        for (int q = 0; q < mem; ++q) {
            if (n_add) n_add[p + q] = add ? na[u] : n_add_from_pof(pof[u]);
            if (pof_mant) pof_mant[p + q] = pof[u].m;
            if (pof_exp) pof_exp[p + q] = (int)pof[u].e;
        }
    }
    auto fin = insert_copies(units, na);
    int len = 0;
    for (auto &u : fin) len += u.kind == UNIT_PAIR ? 2 : 1;
    if (d_eff) *d_eff = len;
    if (re_out && im_out) {
        if (cap < len) {
            set_error("pp_add_roots: capacity too small");
            return PP_EINVAL;
        }
        int o = 0;
        for (auto &u : fin) {
            re_out[o] = u.re;
            im_out[o++] = u.im;
            if (u.kind == UNIT_PAIR) {
                re_out[o] = u.re;
                im_out[o++] = -u.im;
            }
        }
    }
    return PP_OK;
}

pp_status pp_poly_from_roots(int d, const double *re, const double *im, int flags, pp_poly *out) {
    if (d <= 0 || !re || !im || !out) {
        set_error("pp_poly_from_roots: bad argument");
        return PP_EINVAL;
    }
    for (int i = 0; i < d; ++i) {
        if (!std::isfinite(re[i]) || !std::isfinite(im[i])) {
            set_error("pp_poly_from_roots: non-finite root");
            return PP_EINVAL;
        }
        if (re[i] == 0.0 && im[i] == 0.0) {
            set_error("pp_poly_from_roots: zero root");
            return PP_ESINGULAR;
        }
    }
    auto *p = new (std::nothrow) pp_poly_s();
    if (!p) return PP_ENOMEM;
    if (flags & PP_ROOTS_KEEP_ORDER) {
        std::vector<Unit> units;
        std::vector<int> pos;
        if (!units_of(d, re, im, units, pos)) {
            delete p;
            return PP_EINVAL;
        }
        p->plan.leja_re.assign(re, re + d);
        p->plan.leja_im.assign(im, im + d);
        p->plan.pof = pof_values(d, re, im, units, pos);
        p->plan.n_add.assign(units.size(), 0);
        p->plan.units = units;
        p->plan.d = d;
        p->plan.d_eff = d;
        p->plan.n_added = 0;
    } else {
        int st = plan_roots(d, re, im, (flags & PP_ROOTS_ADD) != 0, p->plan);
        if (st != PP_OK) {
            delete p;
            return (pp_status)st;
        }
    }
    p->theta_re.assign(re, re + d);
    p->theta_im.assign(im, im + d);
    p->finalize();
    *out = p;
    return PP_OK;
}

pp_status pp_poly_roots(pp_poly p, int which, int cap, double *re, double *im, int *len, int *d_orig,
                        int *n_added) {
    if (!p || which < 0 || which > 3 || (which == PP_ROOTS_INNER && !p->inner)) {
        set_error("pp_poly_roots: bad argument (PP_ROOTS_INNER needs a composite polynomial)");
        return PP_EINVAL;
    }
    if (d_orig) *d_orig = p->plan.d;
    if (n_added) *n_added = p->plan.n_added;
    std::vector<double> r, i;
    if (which == PP_ROOTS_FINAL || which == PP_ROOTS_INNER) {
        const pp_poly_s *q = which == PP_ROOTS_INNER ? p->inner.get() : p;
        for (auto &u : q->plan.units) {
            r.push_back(u.re);
            i.push_back(u.im);
            if (u.kind == UNIT_PAIR) {
                r.push_back(u.re);
                i.push_back(-u.im);
            }
        }
    } else if (which == PP_ROOTS_THETA) {
        r = p->theta_re;
        i = p->theta_im;
    } else {
        r = p->plan.leja_re;
        i = p->plan.leja_im;
    }
    if (len) *len = (int)r.size();
    if (re && im) {
        if (cap < (int)r.size()) {
            set_error("pp_poly_roots: capacity too small");
            return PP_EINVAL;
        }
        std::copy(r.begin(), r.end(), re);
        std::copy(i.begin(), i.end(), im);
    }
    return PP_OK;
}

void pp_poly_destroy(pp_poly p) { delete p; }

}  // extern "C"
