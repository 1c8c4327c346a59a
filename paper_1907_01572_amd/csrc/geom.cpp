// Analytic macro-element maps and their Jacobians (Sec. II.A.1, Eq. Phi_e; Sec. II.A.5,
// Eq. Jacobian; Sec. III.C, Eq. inverse_mapping and the cubed-sphere macro-mesh): the host
// entry to the maps shared with the device kernels.
#include "host.hpp"
#include "maps.hpp"

namespace hpdg {

void macro_eval(const Macro& M, const double xi[3], double zc, double x[3], double J[3][3]) {
  macro_map(M.kind, M.par, xi, zc, x, J);
}

}  // namespace hpdg
