// kernel_common.hpp -- device helpers shared by the step and adjoint kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "layout.hpp"

namespace arbmi {
namespace dev {

// x / (exp(x) - 1) with its removable singularity at 0
__device__ inline double exprelr(double x) { return (1.0 + x == 1.0) ? 1.0 : x / expm1(x); }

// d/dx of x / (exp(x) - 1); a short series near the removable singularity
__device__ inline double exprelr_dx(double x) {
    if (fabs(x) < 1e-4) return -0.5 + x * (1.0 / 6.0) - x * x * x * (1.0 / 180.0);
    const double em = expm1(x);
    return (em - x * (em + 1.0)) / (em * em);
}

// textbook Hodgkin-Huxley rates (1/ms) at 6.3 C, V in mV
struct Rates {
    double am, bm, ah, bh, an, bn;
};
__device__ inline Rates hh_rates(double v) {
    Rates r;
    r.am = exprelr(-(v + 40.0) * 0.1);
    r.bm = 4.0 * exp(-(v + 65.0) * (1.0 / 18.0));
    r.ah = 0.07 * exp(-(v + 65.0) * 0.05);
    r.bh = 1.0 / (exp(-(v + 35.0) * 0.1) + 1.0);
    r.an = 0.1 * exprelr(-(v + 55.0) * 0.1);
    r.bn = 0.125 * exp(-(v + 65.0) * (1.0 / 80.0));
    return r;
}

// The rates of hh_rates one at a time, with the same expressions (so the
// same values), for spreading them over threads: the four built on exp
// (w = 0..3: bm, ah, bh, bn) and the two built on exprelr (w = 0, 1: am, an).
__device__ inline double hh_rate_exp(int w, double v) {
    const double d = (w == 2) ? 35.0 : 65.0;
    const double k = (w == 0) ? (1.0 / 18.0) : (w == 1) ? 0.05 : (w == 2) ? 0.1 : (1.0 / 80.0);
    const double e = exp(-(v + d) * k);
    if (w == 2) return 1.0 / (e + 1.0);
    return ((w == 0) ? 4.0 : (w == 1) ? 0.07 : 0.125) * e;
}
__device__ inline double hh_rate_exprelr(int w, double v) {
    const double r = exprelr(-(v + (w ? 55.0 : 40.0)) * 0.1);
    return w ? 0.1 * r : r;
}

// exact update of a gate obeying x' = a(1-x) - b x at fixed V over dt
__device__ inline double gate_step(double x, double a, double b, double dt) {
    const double s = a + b;
    const double xinf = a / s;
    return xinf + (x - xinf) * exp(-dt * s);
}

// this thread's position in round R (0 .. w-1), or -1 if it has no branch
__device__ inline int round_index(const RoundDesc& R, int tid) {
    const int i = tid - R.t0;
    return (i >= 0 && i < R.w) ? i : -1;
}

// this thread's task in round R, or an empty task (len 0)
__device__ inline TaskDesc load_task(const TaskDesc* s_tk, const RoundDesc& R, int tid) {
    const int i = round_index(R, tid);
    if (i >= 0) return s_tk[R.task0 + i];
    return TaskDesc{0, -1, 0, 0};
}

}  // namespace dev
}  // namespace arbmi
