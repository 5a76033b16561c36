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

// 1/d from the hardware's approximate reciprocal and two Newton steps
// (within an ulp or so of the rounded quotient; d positive and normal).
__device__ inline double recip(double d) {
    double y = __builtin_amdgcn_rcp(d);
    y = fma(y, fma(-d, y, 1.0), y);
    y = fma(y, fma(-d, y, 1.0), y);
    return y;
}

// The per-gate constants go through an empty asm so that the compiler does
// not specialise the code below for each gate.
__device__ inline double opaque(double x) {
    asm volatile("" : "+v"(x));
    return x;
}

// One gate of an hh instance (w = 0, 1, 2: m, h, n) advanced over a step of
// length dt at fixed V, by the exact update of gate_step with the rates of
// hh_rates, for giving each gate its own thread.  Each rate is formed as a
// quotient, alpha = na/da and beta = nb/db (da = e^xa - 1 for the exprelr
// rates, db = e^xb + 1 for beta_h, 1 otherwise), so alpha + beta = p/q and
// x_inf = alpha/(alpha + beta) = na db/p with p = na db + nb da, q = da db,
// and one reciprocal of p q gives both.  e^x and e^x - 1 come from exp_pair
// (a shorter dependency chain than the library's, within 2 ulp of it).
// The gate's constants are chosen once (hh_gate_consts, kept in registers
// across steps); every thread runs the same straight-line code.
struct HHGate {
    double oa, sa;  // alpha's argument -(v + oa) sa
    double ob, sb;  // beta's argument -(v + ob) sb
    double ka, kb;  // factors of alpha and beta
    bool h;         // the h gate: alpha = ka e^xa, beta = 1/(e^xb + 1)
};
__device__ inline HHGate hh_gate_consts(int w) {
    HHGate c;
    c.oa = opaque((w == 0) ? 40.0 : (w == 1) ? 65.0 : 55.0);
    c.sa = opaque((w == 1) ? 0.05 : 0.1);
    c.ob = opaque((w == 1) ? 35.0 : 65.0);
    c.sb = opaque((w == 0) ? (1.0 / 18.0) : (w == 1) ? 0.1 : (1.0 / 80.0));
    c.ka = opaque((w == 0) ? 1.0 : (w == 1) ? 0.07 : 0.1);
    c.kb = opaque((w == 0) ? 4.0 : 0.125);
    c.h = w == 1;
    return c;
}
__device__ inline double hh_gate_step(const HHGate& c, double v, double x, double dt) {
    const double xa = -(v + c.oa) * c.sa;
    const ExpPair pa = exp_pair(xa);
    const double xb = -(v + c.ob) * c.sb;
    const double eb = exp_pair(xb).e;
    const bool tiny = 1.0 + xa == 1.0;  // exprelr's removable singularity: alpha_m = 1, alpha_n = 0.1
    const double na = c.ka * (c.h ? pa.e : tiny ? 1.0 : xa);
    const double da = (c.h || tiny) ? 1.0 : pa.em1;
    const double nb = c.h ? 1.0 : c.kb * eb;
    const double db = c.h ? eb + 1.0 : 1.0;
    const double p = na * db + nb * da;
    const double q = da * db;
    const double r = recip(p * q);
    const double s = p * (p * r);  // alpha + beta
    const double xinf = (na * db) * (q * r);
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
