// Host-side building blocks of the polynomial preconditioner (internal).
//
// Everything here runs on the CPU in IEEE binary64 with no contraction of
// multiply-adds (the file is compiled with -ffp-contract=off), so root
// ordering and root counts are reproducible bit for bit.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace ppg {

enum UnitKind : int { UNIT_REAL = 0, UNIT_PAIR = 1 };

// A factor of pi: a real root theta (im = 0) or a conjugate pair a +/- bi
// (folded into one real quadratic factor, eq. 2.2).
struct Unit {
    int kind;
    double re;
    double im;  // > 0 for a pair
};

// Running product kept as mantissa in [0.5, 1) and binary exponent.
struct MantExp {
    double m;
    long e;
};

void set_error(const std::string &msg);

// Francis double-shift QR on an upper Hessenberg matrix (column-major,
// leading dimension ld). Returns false if the iteration does not converge.
bool hessenberg_eig(int k, const double *h, int ld, double *re, double *im);

// Harmonic Ritz values (Algorithm 4 step 1b). Returns 0, or -4 (singular).
int harmonic_ritz(int k, const double *hbar, bool breakdown, double *re, double *im);

// Modified Leja permutation of the roots. Returns false on unpaired complex roots.
bool leja_order(int d, const double *re, const double *im, int *perm);

// Units of a Leja-ordered root list; false if pairs are not adjacent conjugates.
bool units_of(int d, const double *re, const double *im, std::vector<Unit> &units,
              std::vector<int> &pos);

// pof per unit (Algorithm 2 step 2).
std::vector<MantExp> pof_values(int d, const double *re, const double *im,
                                const std::vector<Unit> &units, const std::vector<int> &pos);

// Copies per unit (Algorithm 2 step 3).
int n_add_from_pof(const MantExp &pof);

// Insert copies (Algorithm 2 step 3): returns the final unit list.
std::vector<Unit> insert_copies(const std::vector<Unit> &units, const std::vector<int> &n_add);

// Whole ordering + root adding from raw roots. Returns 0 or a negative status.
struct RootPlan {
    std::vector<double> leja_re, leja_im;  // ordered original roots
    std::vector<Unit> units;               // final unit list (with copies)
    std::vector<int> n_add;                // per Leja unit
    std::vector<MantExp> pof;              // per Leja unit
    int d = 0, d_eff = 0, n_added = 0;
};
int plan_roots(int d, const double *re, const double *im, bool add, RootPlan &out);

// Givens-rotation least squares for GMRES: incremental QR of Hbar.
struct GivensLS {
    int m = 0;
    std::vector<double> R;   // (m+1) x m column-major, rotated Hessenberg
    std::vector<double> c, s, g;
    int k = 0;               // columns added
    void reset(int m_, double beta);
    // Add column j (length j+2) of Hbar; returns |g[j+1]| (shortcut residual).
    double add_column(const double *h);
    // Solve R z = g for the first k columns.
    void solve(double *z) const;
};

}  // namespace ppg
