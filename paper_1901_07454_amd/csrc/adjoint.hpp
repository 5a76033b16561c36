// adjoint.hpp -- discrete adjoint of the step (gradients of a soma-trace loss).
#pragma once
#include <stdint.h>

namespace arbmi {
struct Sim;
int grad_forward(Sim* s, int64_t n_steps, int32_t ckpt_every, double* trace_dev);
int grad_backward(Sim* s, const double* dL_dtrace_dev, double* dL_dtheta_dev);
void grad_release(Sim* s);
}  // namespace arbmi
