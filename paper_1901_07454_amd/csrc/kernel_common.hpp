// kernel_common.hpp -- device helpers shared by the step and adjoint kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "fastexp.hpp"
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

// The two rates of one gate of hh_rates (w = 0, 1, 2: m, h, n), with the
// same expressions, for giving each gate its own thread; e^x and e^x - 1 come
// from exp_pair (a shorter dependency chain than the library's, within 2 ulp
// of it).  Both candidate forms of alpha (exprelr-based for m and n,
// exp-based for h) come from the one exp_pair of its argument and one is
// kept, so every thread runs the same straight-line code; the per-gate
// constants go through an empty asm so that the compiler does not specialise
// the code for each constant.
__device__ inline double opaque(double x) {
    asm volatile("" : "+v"(x));
    return x;
}
__device__ inline void hh_gate_rates(int w, double v, double& alpha, double& beta) {
    const double xa = -(v + opaque((w == 0) ? 40.0 : (w == 1) ? 65.0 : 55.0)) * opaque((w == 1) ? 0.05 : 0.1);
    const ExpPair pa = exp_pair(xa);
    const double er = (1.0 + xa == 1.0) ? 1.0 : xa / pa.em1;  // exprelr(xa)
    alpha = (w == 1) ? 0.07 * pa.e : (w == 2) ? 0.1 * er : er;
    const double xb = -(v + opaque((w == 1) ? 35.0 : 65.0)) *
                      opaque((w == 0) ? (1.0 / 18.0) : (w == 1) ? 0.1 : (1.0 / 80.0));
    const double eb = exp_pair(xb).e;
    beta = (w == 1) ? 1.0 / (eb + 1.0) : ((w == 0) ? 4.0 : 0.125) * eb;
}

// gate_step with e^x from exp_pair
__device__ inline double gate_step_pair(double x, double a, double b, double dt) {
    const double s = a + b;
    const double xinf = a / s;
    return xinf + (x - xinf) * exp_pair(-dt * s).e;
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
