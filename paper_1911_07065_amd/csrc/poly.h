// The polynomial object behind the opaque pp_poly handle, and the chain
// programs derived from its root list (internal).
#pragma once

#include <memory>
#include <vector>

#include "host_core.h"

namespace ppg {

// Symbolic buffers a chain step reads or writes.
enum Buf : int { B_NONE = -1, B_IN = 0, B_OUT = 1, B_P0 = 2, B_P1 = 3, B_T = 4 };

// One fused launch: w = a0*(A in) + a1*in + a2*aux;
//   if acc: acc = (acc_init ? 0 : acc) + b0*in + b1*w;
//   out = fin ? IN - w : w.
// spmv == 0 marks an elementwise step without the sparse product (a0 unused).
struct Step {
    int spmv;
    int in, aux, out, acc;
    int acc_init;
    int fin;
    double a0, a1, a2, b0, b1;
};

unsigned long long next_poly_id();

// phi(A)v by Algorithm 1 (or pi(A)v when want_pi): d_eff sparse products.
std::vector<Step> program_phi(const std::vector<Unit> &units, bool want_pi);
// p(A)v by Algorithm 3: d_eff - 1 sparse products; the last real unit's
// contribution is folded into the step before it. Result lands in B_OUT.
std::vector<Step> program_p(const std::vector<Unit> &units);

}  // namespace ppg

struct pp_poly_s {
    unsigned long long id = 0;  // unique per polynomial (keys device-side caches)
    ppg::RootPlan plan;
    std::vector<double> theta_re, theta_im;  // raw harmonic Ritz values
    int breakdown = 0;
    std::vector<ppg::Step> prog_p, prog_phi, prog_pi;
    // Composite (double) polynomial phi2(phi1(A)): this object holds phi2's
    // roots (in the variable of phi1(A)) and inner is phi1 (section 6).
    std::shared_ptr<const pp_poly_s> inner;
    void finalize() {
        id = ppg::next_poly_id();
        prog_p = ppg::program_p(plan.units);
        prog_phi = ppg::program_phi(plan.units, false);
        prog_pi = ppg::program_phi(plan.units, true);
    }
};
