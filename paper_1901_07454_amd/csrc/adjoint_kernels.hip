// adjoint_kernels.hip -- discrete adjoint of the step on gfx950.
//
// The paper computes no gradients; this differentiates exactly the forward
// scheme of kernels.hip.  With A = C/dt + L (symmetric, step-invariant), one
// forward step n is
//   g~ = g^n + events(n)                      (fixed inputs)
//   A V^{n+1} = (C/dt) V^n - I(V^n, x^n, g~; theta)
//   x^{n+1} = Phi(x^n, V^{n+1})  for the hh gates x in {m, h, n}.
// Going backwards with lambda_V = dL/dV^{n+1} (all later dependencies
// included except the gate update of this step) and lambda_x = dL/dx^{n+1}:
//   u = lambda_V + sum_x (dPhi_x/dV^{n+1}) lambda_x
//   A w = u                                   (same Hines solve, A = A^T)
//   lambda_V <- (C/dt - dI/dV) w   (+ dL/dtrace of the previous step)
//   lambda_x <- (dPhi_x/dx) lambda_x - (dI/dx) w
//   dL/dtheta -= (dI/dtheta)^T w
// One workgroup runs one pack backwards through a checkpoint segment; the
// forward states of the segment were recorded by a recompute pass.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "adjoint_kernels.hpp"
#include "kernel_common.hpp"

namespace arbmi {

namespace {

using namespace dev;

struct GateD {
    double E;      // dPhi/dx = exp(-dt (a + b))
    double dPhi;   // dPhi/dV at V^{n+1}
};

// rates a(v), b(v), their derivatives, and the gate update's sensitivities
__device__ inline GateD gate_sens(double x0, double a, double b, double da, double db, double dt) {
    const double s = a + b;
    const double E = exp(-dt * s);
    const double xinf = a / s;
    const double dxinf = (da * b - a * db) / (s * s);
    GateD g;
    g.E = E;
    g.dPhi = dxinf * (1.0 - E) + (x0 - xinf) * E * (-dt * (da + db));
    return g;
}

constexpr int CH = 8;

template <int T>
__global__ void __launch_bounds__(T) adjoint_kernel(AdjArgs a) {
    extern __shared__ double lds[];
    const int p = blockIdx.x;
    const PackDesc pk = a.pk[p];
    const int tid = threadIdx.x;
    const int ns = pk.nslot;

    double* sL = lds;            // lambda_V
    double* sW = sL + ns;        // solve workspace
    double* sPa1 = sW + ns;      // sum w V   (pas gradient)
    double* sPa0 = sPa1 + ns;    // sum w     (pas gradient)
    double* sLm = sPa0 + ns;     // lambda_m, lambda_h, lambda_n
    double* sLh = sLm + pk.nhh;
    double* sLn = sLh + pk.nhh;
    double* sGna = sLn + pk.nhh; // hh gradient accumulators
    double* sGk = sGna + pk.nhh;
    RoundDesc* s_rd = reinterpret_cast<RoundDesc*>(sGk + pk.nhh);
    TaskDesc* s_tk = reinterpret_cast<TaskDesc*>(s_rd + pk.nrd);
    NlDesc* s_nl = reinterpret_cast<NlDesc*>(s_tk + pk.ntk);
    int32_t* s_ch = reinterpret_cast<int32_t*>(s_nl + pk.nnl);

    const double* gA = a.alpha + pk.slot0;
    const double* gF = a.F + pk.slot0;
    const double* gD = a.invd + pk.slot0;

    for (int i = tid; i < ns; i += T) {
        sL[i] = a.lamV[pk.slot0 + i];
        sW[i] = 0.0;
        sPa1[i] = 0.0;
        sPa0[i] = 0.0;
    }
    for (int i = tid; i < pk.nhh; i += T) {
        sLm[i] = a.lamM[pk.hh0 + i];
        sLh[i] = a.lamH[pk.hh0 + i];
        sLn[i] = a.lamN[pk.hh0 + i];
        sGna[i] = 0.0;
        sGk[i] = 0.0;
    }
    for (int i = tid; i < pk.nrd; i += T) s_rd[i] = a.rd[pk.rd0 + i];
    for (int i = tid; i < pk.ntk; i += T) s_tk[i] = a.tk[pk.tk0 + i];
    for (int i = tid; i < pk.nnl; i += T) s_nl[i] = a.nl[pk.nl0 + i];
    for (int i = tid; i < pk.nch; i += T) s_ch[i] = a.ch_slot[pk.ch0 + i];
    const int soma = (tid < pk.ncell) ? a.pc_soma[pk.cell0 + tid] : -1;
    const int gid = (tid < pk.ncell) ? a.pc_gid[pk.cell0 + tid] : -1;
    __syncthreads();

    for (int s = a.nsteps - 1; s >= 0; --s) {
        const int64_t n = a.step0 + s;  // reversing step n -> n+1
        const double* V0 = a.rec_V + int64_t(s) * a.n_slots_total + pk.slot0;
        const double* V1 = V0 + a.n_slots_total;
        const double* M0 = a.rec_m + int64_t(s) * a.n_hh_total + pk.hh0;
        const double* H0 = a.rec_h + int64_t(s) * a.n_hh_total + pk.hh0;
        const double* N0 = a.rec_n + int64_t(s) * a.n_hh_total + pk.hh0;
        const double* G0 = a.rec_g + int64_t(s) * a.n_syn_total + pk.syn0;

        // loss term dL/dV_soma^{n+1}
        if (soma >= 0) sL[soma] += a.dLdtrace[int64_t(gid) * a.trace_len + (n - a.trace_step0)];
        __syncthreads();

        // u = lambda_V (+ gate-update terms at hh CVs); lambda_x *= dPhi/dx
        for (int i = tid; i < ns; i += T) sW[i] = sL[i];
        __syncthreads();
        for (int j = tid; j < pk.nnl; j += T) {
            const NlDesc d = s_nl[j];
            if (d.hh < 0) continue;
            const int q = d.hh;
            const double v = V1[d.slot];
            // rates and their derivatives at V^{n+1}
            const double xm = -(v + 40.0) * 0.1, xn = -(v + 55.0) * 0.1;
            const double am = exprelr(xm), dam = -0.1 * exprelr_dx(xm);
            const double ebm = exp(-(v + 65.0) * (1.0 / 18.0));
            const double bm = 4.0 * ebm, dbm = -(4.0 / 18.0) * ebm;
            const double eah = exp(-(v + 65.0) * 0.05);
            const double ah = 0.07 * eah, dah = -(0.07 / 20.0) * eah;
            const double u = exp(-(v + 35.0) * 0.1);
            const double bh = 1.0 / (u + 1.0), dbh = 0.1 * u / ((1.0 + u) * (1.0 + u));
            const double an = 0.1 * exprelr(xn), dan = -0.01 * exprelr_dx(xn);
            const double ebn = exp(-(v + 65.0) * (1.0 / 80.0));
            const double bn = 0.125 * ebn, dbn = -(0.125 / 80.0) * ebn;
            const GateD gm = gate_sens(M0[q], am, bm, dam, dbm, a.dt);
            const GateD gh = gate_sens(H0[q], ah, bh, dah, dbh, a.dt);
            const GateD gn = gate_sens(N0[q], an, bn, dan, dbn, a.dt);
            sW[d.slot] += gm.dPhi * sLm[q] + gh.dPhi * sLh[q] + gn.dPhi * sLn[q];
            sLm[q] *= gm.E;
            sLh[q] *= gh.E;
            sLn[q] *= gn.E;
        }
        __syncthreads();

        // A w = u: elimination (deepest rounds first) then substitution
        {
            RoundDesc R = s_rd[0];
            TaskDesc t = load_task(s_tk, R, tid);
            for (int r = 0; r < pk.nrd; ++r) {
                RoundDesc Rn = R;
                TaskDesc tn = t;
                if (r + 1 < pk.nrd) {
                    Rn = s_rd[r + 1];
                    tn = load_task(s_tk, Rn, tid);
                }
                if (t.len > 0) {
                    const int base = R.slot0 + (tid - R.t0);
                    const int w = R.w;
                    double csum = 0.0;
                    for (int c = 0; c < t.nch; ++c) {
                        const int cs = s_ch[t.ch0 + c];
                        csum += gF[cs] * sW[cs];
                    }
                    double acc = 0.0, fprev = 0.0;
                    for (int k0 = t.len - 1; k0 >= 0; k0 -= CH) {
                        double tv[CH], fv[CH];
#pragma unroll
                        for (int j = 0; j < CH; ++j) {
                            const int sl = base + max(k0 - j, 0) * w;
                            tv[j] = sW[sl];
                            fv[j] = gF[sl];
                        }
#pragma unroll
                        for (int j = 0; j < CH; ++j) {
                            const int k = k0 - j;
                            if (k >= 0) {
                                acc = (k == t.len - 1) ? tv[j] - csum : tv[j] - fprev * acc;
                                fprev = fv[j];
                                sW[base + k * w] = acc;
                            }
                        }
                    }
                }
                __syncthreads();
                R = Rn;
                t = tn;
            }
        }
        {
            RoundDesc R = s_rd[pk.nrd - 1];
            TaskDesc t = load_task(s_tk, R, tid);
            for (int r = pk.nrd - 1; r >= 0; --r) {
                RoundDesc Rn = R;
                TaskDesc tn = t;
                if (r > 0) {
                    Rn = s_rd[r - 1];
                    tn = load_task(s_tk, Rn, tid);
                }
                if (t.len > 0) {
                    const int base = R.slot0 + (tid - R.t0);
                    const int w = R.w;
                    double x = (t.par >= 0) ? sW[t.par] : 0.0;
                    for (int k0 = 0; k0 < t.len; k0 += CH) {
                        double rv[CH], dv[CH], fv[CH];
#pragma unroll
                        for (int j = 0; j < CH; ++j) {
                            const int sl = base + min(k0 + j, t.len - 1) * w;
                            rv[j] = sW[sl];
                            dv[j] = gD[sl];
                            fv[j] = gF[sl];
                        }
#pragma unroll
                        for (int j = 0; j < CH; ++j) {
                            const int k = k0 + j;
                            if (k < t.len) {
                                x = rv[j] * dv[j] - fv[j] * x;
                                sW[base + k * w] = x;
                            }
                        }
                    }
                }
                __syncthreads();
                R = Rn;
                t = tn;
            }
        }

        // lambda_V = (C/dt - G_lin) w - (nonlinear dI/dV) w; parameter terms
        for (int i = tid; i < ns; i += T) {
            const double w = sW[i];
            sL[i] = gA[i] * w;
            sPa1[i] += w * V0[i];
            sPa0[i] += w;
        }
        __syncthreads();
        for (int j = tid; j < pk.nnl; j += T) {
            const NlDesc d = s_nl[j];
            const double w = sW[d.slot];
            const double v = V0[d.slot];
            double dIdV = 0.0;
            if (d.hh >= 0) {
                const int q = d.hh;
                const double m = M0[q], h = H0[q], g = N0[q];
                const double gna = a.hh_gna[pk.hh0 + q], gk = a.hh_gk[pk.hh0 + q];
                const double m3h = m * m * m * h, n4 = g * g * g * g;
                dIdV += gna * m3h + gk * n4;
                sLm[q] -= gna * 3.0 * m * m * h * (v - kENa) * w;
                sLh[q] -= gna * m * m * m * (v - kENa) * w;
                sLn[q] -= gk * 4.0 * g * g * g * (v - kEK) * w;
                sGna[q] -= m3h * (v - kENa) * w;
                sGk[q] -= n4 * (v - kEK) * w;
            }
            for (int k = 0; k < d.nsyn; ++k) dIdV += G0[d.syn0 + k];
            sL[d.slot] -= dIdV * w;
        }
        __syncthreads();
    }

    for (int i = tid; i < ns; i += T) {
        a.lamV[pk.slot0 + i] = sL[i];
        a.accP1[pk.slot0 + i] += sPa1[i];
        a.accP0[pk.slot0 + i] += sPa0[i];
    }
    for (int i = tid; i < pk.nhh; i += T) {
        a.lamM[pk.hh0 + i] = sLm[i];
        a.lamH[pk.hh0 + i] = sLh[i];
        a.lamN[pk.hh0 + i] = sLn[i];
        a.accNa[pk.hh0 + i] += sGna[i];
        a.accK[pk.hh0 + i] += sGk[i];
    }
}

// dL/dtheta[r] = (gNa, gK, g_pas) for region r from the per-CV sums:
// each membrane piece (CV slot, area) of the region contributes 10 * area
// (S/cm^2 x um^2 -> nS) times the CV's sensitivity.
__global__ void grad_reduce_kernel(GradReduceArgs a) {
    const int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (r >= a.n_reg) return;
    double gna = 0.0, gk = 0.0, gpas = 0.0;
    const uint32_t mech = a.reg_mech[r];
    const double epas = a.reg_epas[r];
    for (int64_t k = a.rp_off[r]; k < a.rp_off[r + 1]; ++k) {
        const double a10 = 10.0 * a.rp_area[k];
        const int64_t slot = a.rp_slot[k];
        const int64_t hh = a.rp_hh[k];
        if ((mech & 1u) && hh >= 0) {
            gna += a10 * a.accNa[hh];
            gk += a10 * a.accK[hh];
        }
        if (mech & 2u) gpas += a10 * (epas * a.accP0[slot] - a.accP1[slot]);
    }
    a.out[3 * r + 0] = gna;
    a.out[3 * r + 1] = gk;
    a.out[3 * r + 2] = gpas;
}

__global__ void copy_parts_kernel(CopyList c) {
    const int q = blockIdx.y;
    const int64_t n = c.words[q];
    const uint32_t* src = c.src[q];
    uint32_t* dst = c.dst[q];
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
        dst[i] = src[i];
}

template <int T>
hipError_t launch_adj(const AdjArgs& a, int lds, int n_packs, hipStream_t st) {
    hipLaunchKernelGGL((adjoint_kernel<T>), dim3(n_packs), dim3(T), lds, st, a);
    return hipGetLastError();
}

}  // namespace

hipError_t prepare_adjoint_kernels(int lds_max) {
    const void* fns[] = {reinterpret_cast<const void*>(&adjoint_kernel<64>),
                         reinterpret_cast<const void*>(&adjoint_kernel<128>),
                         reinterpret_cast<const void*>(&adjoint_kernel<256>)};
    for (const void* f : fns) {
        hipFuncAttributes at{};
        if (hipFuncGetAttributes(&at, f) != hipSuccess) continue;
        const int allowed = lds_max - int(at.sharedSizeBytes);
        if (allowed > 0) (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, allowed);
        (void)hipGetLastError();
    }
    return hipSuccess;
}

hipError_t launch_adjoint(const AdjArgs& a, int block_threads, int lds_bytes, int n_packs, hipStream_t st) {
    switch (block_threads) {
        case 64: return launch_adj<64>(a, lds_bytes, n_packs, st);
        case 128: return launch_adj<128>(a, lds_bytes, n_packs, st);
        case 256: return launch_adj<256>(a, lds_bytes, n_packs, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_copy_parts(const CopyList& c, hipStream_t st) {
    if (c.n <= 0) return hipSuccess;
    if (c.n > kCopyParts) return hipErrorInvalidValue;
    int64_t most = 0;
    for (int q = 0; q < c.n; ++q) most = c.words[q] > most ? c.words[q] : most;
    const unsigned nb = unsigned(std::min<int64_t>(1024, std::max<int64_t>(1, (most + 255) / 256)));
    hipLaunchKernelGGL(copy_parts_kernel, dim3(nb, unsigned(c.n)), dim3(256), 0, st, c);
    return hipGetLastError();
}

hipError_t launch_grad_reduce(const GradReduceArgs& a, hipStream_t st) {
    if (a.n_reg <= 0) return hipSuccess;
    hipLaunchKernelGGL(grad_reduce_kernel, dim3(unsigned((a.n_reg + 255) / 256)), dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace arbmi
