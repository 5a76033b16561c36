// adjoint.cpp -- host side of the discrete adjoint.
#include "adjoint.hpp"

#include "sim.hpp"

namespace arbmi {

int grad_forward(Sim* s, int64_t n_steps, int32_t ckpt_every, double* trace_dev) {
    (void)s; (void)n_steps; (void)ckpt_every; (void)trace_dev;
    return set_error(ARB_ESTATE, "gradients are not available in this build");
}

int grad_backward(Sim* s, const double* dL_dtrace_dev, double* dL_dtheta_dev) {
    (void)s; (void)dL_dtrace_dev; (void)dL_dtheta_dev;
    return set_error(ARB_ESTATE, "arb_grad_backward before arb_grad_forward");
}

void grad_release(Sim* s) { (void)s; }

}  // namespace arbmi
