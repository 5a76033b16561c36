// kernels.hip -- HIP kernels of the cell stepper for gfx950 (CDNA4).
//
// One workgroup advances one pack of cells through every step of an epoch
// (cells are independent within an epoch because no spike can arrive sooner
// than the minimum delay, Sec. II).  The pack's voltages live in LDS for the
// whole launch; the per-CV step coefficients are staged in LDS too
// (coefficient mode 1) or re-read from global memory every step (mode 2).
// A step (Sec. II operator splitting) is:
//   A  events due at this step: g_syn += w
//   B  point and nonlinear currents at V^n (hh, expsyn, clamps) -> R
//   C  elimination of the implicit-Euler right-hand side, deepest branch
//      rounds first: each thread walks its branch from the distal end,
//      rhs = alpha V + beta + R, minus F x (eliminated rhs) of the children
//   D  substitution, shallowest rounds first: x = rhs' / d' - F x_parent
//   E  gates and synapse decay with V^{n+1}; soma threshold test; probes
// The matrix is step-invariant (the membrane current is explicit), so its
// factorisation (F, 1/d') is computed once on the host.
#include <hip/hip_runtime.h>

#include "kernel_common.hpp"
#include "kernels.hpp"

namespace arbmi {

namespace {

using namespace dev;

constexpr int CH = 8;  // CVs of a branch staged in registers at a time

template <int T, bool CL>
__global__ void __launch_bounds__(T) step_kernel(StepArgs a) {
    extern __shared__ double lds[];
    const int p = blockIdx.x + a.pack0;
    const PackDesc pk = a.pk[p];
    const int tid = threadIdx.x;
    const int ns = pk.nslot;

    // ---- LDS layout (must match pack_lds_bytes) ----
    double* sV = lds;
    double* sR = sV + ns;
    double* sA = sR + ns;
    double* sB = sA + ns;
    double* sF = sB + ns;
    double* sD = sF + ns;
    double* sg = CL ? sD + ns : sR + ns;
    double* sm = sg + pk.nsyn;
    double* sh = sm + pk.nhh;
    double* sn = sh + pk.nhh;
    double* s_gna = sn + pk.nhh;  // mode 1 only
    double* s_gk = s_gna + pk.nhh;
    double* s_se = s_gk + pk.nhh;
    double* s_sdec = s_se + pk.nsyn;
    RoundDesc* s_rd = reinterpret_cast<RoundDesc*>(CL ? s_sdec + pk.nsyn : sn + pk.nhh);
    TaskDesc* s_tk = reinterpret_cast<TaskDesc*>(s_rd + pk.nrd);
    NlDesc* s_nl = reinterpret_cast<NlDesc*>(s_tk + pk.ntk);
    int32_t* s_ch = reinterpret_cast<int32_t*>(s_nl + pk.nnl);

    const double* gA = a.alpha + pk.slot0;
    const double* gB = a.beta + pk.slot0;
    const double* gF = a.F + pk.slot0;
    const double* gD = a.invd + pk.slot0;
    auto ldA = [&](int i) { if constexpr (CL) return sA[i]; else return gA[i]; };
    auto ldB = [&](int i) { if constexpr (CL) return sB[i]; else return gB[i]; };
    auto ldF = [&](int i) { if constexpr (CL) return sF[i]; else return gF[i]; };
    auto ldD = [&](int i) { if constexpr (CL) return sD[i]; else return gD[i]; };
    const double* g_gna = a.hh_gna + pk.hh0;
    const double* g_gk = a.hh_gk + pk.hh0;
    const double* g_se = a.syn_e + pk.syn0;
    const double* g_sdec = a.syn_decay + pk.syn0;
    auto ldGna = [&](int i) { if constexpr (CL) return s_gna[i]; else return g_gna[i]; };
    auto ldGk = [&](int i) { if constexpr (CL) return s_gk[i]; else return g_gk[i]; };
    auto ldSe = [&](int i) { if constexpr (CL) return s_se[i]; else return g_se[i]; };
    auto ldSdec = [&](int i) { if constexpr (CL) return s_sdec[i]; else return g_sdec[i]; };

    // ---- stage the pack in LDS ----
    for (int i = tid; i < ns; i += T) {
        sV[i] = a.V[pk.slot0 + i];
        sR[i] = 0.0;
        if constexpr (CL) {
            sA[i] = gA[i];
            sB[i] = gB[i];
            sF[i] = gF[i];
            sD[i] = gD[i];
        }
    }
    for (int i = tid; i < pk.nsyn; i += T) {
        sg[i] = a.syn_g[pk.syn0 + i];
        if constexpr (CL) {
            s_se[i] = g_se[i];
            s_sdec[i] = g_sdec[i];
        }
    }
    for (int i = tid; i < pk.nhh; i += T) {
        sm[i] = a.hh_m[pk.hh0 + i];
        sh[i] = a.hh_h[pk.hh0 + i];
        sn[i] = a.hh_n[pk.hh0 + i];
        if constexpr (CL) {
            s_gna[i] = g_gna[i];
            s_gk[i] = g_gk[i];
        }
    }
    for (int i = tid; i < pk.nrd; i += T) s_rd[i] = a.rd[pk.rd0 + i];
    for (int i = tid; i < pk.ntk; i += T) s_tk[i] = a.tk[pk.tk0 + i];
    for (int i = tid; i < pk.nnl; i += T) s_nl[i] = a.nl[pk.nl0 + i];
    for (int i = tid; i < pk.nch; i += T) s_ch[i] = a.ch_slot[pk.ch0 + i];

    // event cursors live in thread 0's registers, with the next key cached
    int64_t step0 = a.step0;
    int32_t bucket = a.bucket;
    if (a.epoch_ptr) {
        const int64_t e = *a.epoch_ptr;
        step0 = e * a.nsteps;
        bucket = int32_t(e % a.n_buckets);
    }
    const int64_t bk_base = (int64_t(bucket) * a.n_packs + p);
    const uint64_t* ev = a.bk_ev + bk_base * a.bk_cap;
    int32_t ncur = 0, nend = 0;
    int64_t xcur = 0;
    uint64_t nkey = ~uint64_t(0);
    int64_t xstep = INT64_MAX;
    if (tid == 0) {
        xcur = a.pk_xcur[p];
        ncur = a.pk_ncur[p];
        const uint32_t c = a.bk_cnt[bk_base];
        nend = int32_t(c < uint32_t(a.bk_cap) ? c : uint32_t(a.bk_cap));
        if (ncur < nend) nkey = ev[ncur];
        if (xcur < pk.xe1) xstep = a.xe_step[xcur];
    }
    const int soma = (tid < pk.ncell) ? a.pc_soma[pk.cell0 + tid] : -1;
    double vold = 0.0;
    __syncthreads();

    for (int s = 0; s < a.nsteps; ++s) {
        const int64_t n = step0 + s;

        // A: events due at the start of step n (network, then external)
        if (tid == 0) {
            while (int64_t(nkey >> 32) == n) {
                const uint32_t r = uint32_t(nkey);
                sg[a.cr_syn[r]] += a.cr_w[r];
                ++ncur;
                nkey = (ncur < nend) ? ev[ncur] : ~uint64_t(0);
            }
            while (xstep == n) {
                sg[a.xe_syn[xcur]] += a.xe_w[xcur];
                ++xcur;
                xstep = (xcur < pk.xe1) ? a.xe_step[xcur] : INT64_MAX;
            }
        }
        __syncthreads();

        if (a.rec_V) {  // state entering the step, for the adjoint
            double* rv = a.rec_V + int64_t(s) * a.n_slots_total + pk.slot0;
            for (int i = tid; i < ns; i += T) rv[i] = sV[i];
            double* rm = a.rec_m + int64_t(s) * a.n_hh_total + pk.hh0;
            double* rh = a.rec_h + int64_t(s) * a.n_hh_total + pk.hh0;
            double* rn = a.rec_n + int64_t(s) * a.n_hh_total + pk.hh0;
            for (int i = tid; i < pk.nhh; i += T) {
                rm[i] = sm[i];
                rh[i] = sh[i];
                rn[i] = sn[i];
            }
            double* rg = a.rec_g + int64_t(s) * a.n_syn_total + pk.syn0;
            for (int i = tid; i < pk.nsyn; i += T) rg[i] = sg[i];
        }

        // B: nonlinear and point currents at V^n, stored as -I in R
        for (int j = tid; j < pk.nnl; j += T) {
            const NlDesc d = s_nl[j];
            const double v = sV[d.slot];
            double I = 0.0;
            if (d.hh >= 0) {
                const int q = d.hh;
                const double m = sm[q], h = sh[q], g = sn[q];
                I += ldGna(q) * (m * m * m * h) * (v - kENa);
                I += ldGk(q) * (g * g * g * g) * (v - kEK);
            }
            for (int k = 0; k < d.nsyn; ++k) {
                const int q = d.syn0 + k;
                I += sg[q] * (v - ldSe(q));
            }
            sR[d.slot] = -I;
        }
        if (soma >= 0) vold = sV[soma];
        if (pk.nic > 0) {  // current clamps, one thread, in (slot, input) order
            __syncthreads();
            if (tid == 0)
                for (int q = pk.ic0; q < pk.ic0 + pk.nic; ++q)
                    if (a.ic_on[q] <= n && n < a.ic_off[q]) sR[a.ic_slot[q]] += a.ic_amp[q];
        }
        __syncthreads();

        // C: elimination, deepest rounds first.  Each thread walks its branch
        // from the distal end in chunks of CH CVs: the chunk's operands are
        // loaded first (unconditional loads at clamped indices, so they issue
        // together), then the dependent recurrence
        // rhs'_k = t_k - F_{k+1} rhs'_{k+1} runs in registers.  The next
        // round's descriptors are fetched while this round works.
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
                        csum += ldF(cs) * sR[cs];
                    }
                    double acc = 0.0, fprev = 0.0;
                    for (int k0 = t.len - 1; k0 >= 0; k0 -= CH) {
                        double tv[CH], fv[CH];
#pragma unroll
                        for (int j = 0; j < CH; ++j) {
                            const int sl = base + max(k0 - j, 0) * w;
                            tv[j] = ldA(sl) * sV[sl] + ldB(sl) + sR[sl];
                            fv[j] = ldF(sl);
                        }
#pragma unroll
                        for (int j = 0; j < CH; ++j) {
                            const int k = k0 - j;
                            if (k >= 0) {
                                acc = (k == t.len - 1) ? tv[j] - csum : tv[j] - fprev * acc;
                                fprev = fv[j];
                                sR[base + k * w] = acc;
                            }
                        }
                    }
                }
                __syncthreads();
                R = Rn;
                t = tn;
            }
        }

        // D: substitution, shallowest rounds first; clears R for the next step
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
                    double x = (t.par >= 0) ? sV[t.par] : 0.0;
                    for (int k0 = 0; k0 < t.len; k0 += CH) {
                        double rv[CH], dv[CH], fv[CH];
#pragma unroll
                        for (int j = 0; j < CH; ++j) {
                            const int sl = base + min(k0 + j, t.len - 1) * w;
                            rv[j] = sR[sl];
                            dv[j] = ldD(sl);
                            fv[j] = ldF(sl);
                        }
#pragma unroll
                        for (int j = 0; j < CH; ++j) {
                            const int k = k0 + j;
                            if (k < t.len) {
                                const int sl = base + k * w;
                                x = rv[j] * dv[j] - fv[j] * x;
                                sV[sl] = x;
                                sR[sl] = 0.0;
                            }
                        }
                    }
                }
                __syncthreads();
                R = Rn;
                t = tn;
            }
        }

        // E: states with V^{n+1}, threshold, probes
        for (int j = tid; j < pk.nnl; j += T) {
            const NlDesc d = s_nl[j];
            if (d.hh >= 0) {
                const int q = d.hh;
                const Rates rt = hh_rates(sV[d.slot]);
                sm[q] = gate_step(sm[q], rt.am, rt.bm, a.dt);
                sh[q] = gate_step(sh[q], rt.ah, rt.bh, a.dt);
                sn[q] = gate_step(sn[q], rt.an, rt.bn, a.dt);
            }
            for (int k = 0; k < d.nsyn; ++k) {
                const int q = d.syn0 + k;
                sg[q] *= ldSdec(q);
            }
        }
        if (soma >= 0) {
            const double vnew = sV[soma];
            if (vold < a.threshold && vnew >= a.threshold) {
                const uint32_t pos = atomicAdd(&a.ctr->sp_count, 1u);
                if (pos < a.sp_cap) {
                    a.sp_gid[pos] = uint32_t(a.pc_gid[pk.cell0 + tid]);
                    a.sp_step[pos] = n + 1;
                    a.sp_t[pos] = (double(n) + (a.threshold - vold) / (vnew - vold)) * a.dt;
                } else {
                    atomicOr(&a.ctr->flags, kFlagSpikeOverflow);
                }
            }
        }
        if (a.trace) {
            const int64_t col = n - a.trace_step0;
            if (col >= 0 && col < a.trace_cap)
                for (int j = tid; j < pk.npr; j += T)
                    a.trace[int64_t(a.pr_id[pk.pr0 + j]) * a.trace_cap + col] = sV[a.pr_slot[pk.pr0 + j]];
        }
        __syncthreads();
    }

    if (a.rec_V) {
        double* rv = a.rec_V + int64_t(a.nsteps) * a.n_slots_total + pk.slot0;
        for (int i = tid; i < ns; i += T) rv[i] = sV[i];
    }
    for (int i = tid; i < ns; i += T) a.V[pk.slot0 + i] = sV[i];
    for (int i = tid; i < pk.nsyn; i += T) a.syn_g[pk.syn0 + i] = sg[i];
    for (int i = tid; i < pk.nhh; i += T) {
        a.hh_m[pk.hh0 + i] = sm[i];
        a.hh_h[pk.hh0 + i] = sh[i];
        a.hh_n[pk.hh0 + i] = sn[i];
    }
    if (tid == 0) {
        a.pk_xcur[p] = xcur;
        a.pk_ncur[p] = ncur;
        if (a.epoch_end) a.bk_cnt[bk_base] = 0u;
    }
}

__global__ void __launch_bounds__(256) sort_buckets_kernel(uint64_t* bk_ev, uint32_t* bk_cnt, int32_t* pk_ncur,
                                                           int32_t cap, int32_t bucket, int32_t n_packs,
                                                           Counters* ctr, const int64_t* epoch_ptr,
                                                           int32_t n_buckets) {
    extern __shared__ uint64_t keys[];
    const int p = blockIdx.x;
    const int tid = threadIdx.x;
    if (epoch_ptr) bucket = int32_t(*epoch_ptr % n_buckets);
    const int64_t base_i = int64_t(bucket) * n_packs + p;
    uint32_t n = bk_cnt[base_i];
    if (tid == 0) pk_ncur[p] = 0;
    if (n > uint32_t(cap)) {
        if (tid == 0) atomicOr(&ctr->flags, kFlagEventOverflow);
        n = uint32_t(cap);
    }
    if (n <= 1) return;
    uint32_t m = 1;
    while (m < n) m <<= 1;
    uint64_t* base = bk_ev + base_i * cap;
    for (uint32_t i = tid; i < m; i += blockDim.x) keys[i] = (i < n) ? base[i] : ~uint64_t(0);
    __syncthreads();
    for (uint32_t k = 2; k <= m; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            for (uint32_t i = tid; i < m; i += blockDim.x) {
                const uint32_t ixj = i ^ j;
                if (ixj > i) {
                    const bool up = (i & k) == 0;
                    const uint64_t x = keys[i], y = keys[ixj];
                    if ((x > y) == up) {
                        keys[i] = y;
                        keys[ixj] = x;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (uint32_t i = tid; i < n; i += blockDim.x) base[i] = keys[i];
}

__global__ void __launch_bounds__(256) exchange_kernel(ExchArgs a) {
    const uint32_t sp_cap = a.sp_cap;
    const int lane = threadIdx.x & 63;
    const int64_t wave = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = (int64_t(gridDim.x) * blockDim.x) >> 6;
    const uint32_t b = a.ctr->sp_exch;
    uint32_t e = a.ctr->sp_count;
    if (e > sp_cap) e = sp_cap;
    for (int64_t i = int64_t(b) + wave; i < int64_t(e); i += nwaves) {
        const uint32_t gid = a.sp_gid[i];
        const int64_t st = a.sp_step[i];
        for (int64_t c = a.out_off[gid] + lane; c < a.out_off[gid + 1]; c += 64) {
            const uint32_t r = a.out_rank[c];
            const int32_t pkk = a.cr_pack[r];
            const int64_t sd = st + a.cr_delay[r];
            const int32_t bk = int32_t((sd / a.epoch_steps) % a.n_buckets);
            const int64_t slot = int64_t(bk) * a.n_packs + pkk;
            const uint32_t pos = atomicAdd(&a.bk_cnt[slot], 1u);
            if (pos < uint32_t(a.bk_cap))
                a.bk_ev[slot * a.bk_cap + pos] = (uint64_t(sd) << 32) | uint64_t(r);
            else
                atomicOr(&a.ctr->flags, kFlagEventOverflow);
        }
    }
}

__global__ void advance_epoch_kernel(int64_t* epoch) { *epoch += 1; }

__global__ void commit_exchange_kernel(Counters* ctr, uint32_t sp_cap) {
    const uint32_t e = ctr->sp_count;
    ctr->sp_exch = e > sp_cap ? sp_cap : e;
}

__global__ void gather_kernel(const double* V, const int64_t* perm, double* dst, int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = V[perm[i]];
}

__global__ void scatter_kernel(double* V, const int64_t* perm, const double* src, int64_t n) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) V[perm[i]] = src[i];
}

template <int T, bool CL>
hipError_t launch_one(const StepArgs& a, int lds, int n_packs, hipStream_t st) {
    hipLaunchKernelGGL((step_kernel<T, CL>), dim3(n_packs), dim3(T), lds, st, a);
    return hipGetLastError();
}

// Allow each kernel the device's LDS minus its own static LDS.  HIP on
// gfx950 accepts launches up to the hardware limit; the attribute is set when
// the runtime supports it and a refusal is not an error here (a launch that
// asks for too much still fails and is reported).
hipError_t allow_lds(const void* fn, int lds_max) {
    hipFuncAttributes at{};
    if (hipFuncGetAttributes(&at, fn) != hipSuccess) return hipSuccess;
    const int allowed = lds_max - int(at.sharedSizeBytes);
    if (allowed > 0) (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, allowed);
    (void)hipGetLastError();
    return hipSuccess;
}

}  // namespace

hipError_t prepare_step_kernels(int max_lds) {
    const void* fns[] = {reinterpret_cast<const void*>(&step_kernel<64, true>),
                         reinterpret_cast<const void*>(&step_kernel<64, false>),
                         reinterpret_cast<const void*>(&step_kernel<128, true>),
                         reinterpret_cast<const void*>(&step_kernel<128, false>),
                         reinterpret_cast<const void*>(&step_kernel<256, true>),
                         reinterpret_cast<const void*>(&step_kernel<256, false>),
                         reinterpret_cast<const void*>(&sort_buckets_kernel)};
    for (const void* f : fns) allow_lds(f, max_lds);
    return prepare_reg_kernels(max_lds);
}

hipError_t launch_step(const StepArgs& a, const LaunchCfg& cfg, int n_packs, hipStream_t st) {
    if (cfg.coef_mode == 3) return launch_reg_step(a, cfg, n_packs, st);
    const bool cl = cfg.coef_mode == 1;
    switch (cfg.block_threads) {
        case 64: return cl ? launch_one<64, true>(a, cfg.lds_bytes, n_packs, st) : launch_one<64, false>(a, cfg.lds_bytes, n_packs, st);
        case 128: return cl ? launch_one<128, true>(a, cfg.lds_bytes, n_packs, st) : launch_one<128, false>(a, cfg.lds_bytes, n_packs, st);
        case 256: return cl ? launch_one<256, true>(a, cfg.lds_bytes, n_packs, st) : launch_one<256, false>(a, cfg.lds_bytes, n_packs, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_sort_buckets(uint64_t* bk_ev, uint32_t* bk_cnt, int32_t* pk_ncur, int32_t bk_cap,
                               int32_t bucket, int32_t n_packs, Counters* ctr, hipStream_t st,
                               const int64_t* epoch_ptr, int32_t n_buckets) {
    int m = 1;
    while (m < bk_cap) m <<= 1;
    hipLaunchKernelGGL(sort_buckets_kernel, dim3(n_packs), dim3(256), size_t(m) * 8, st, bk_ev, bk_cnt, pk_ncur,
                       bk_cap, bucket, n_packs, ctr, epoch_ptr, n_buckets);
    return hipGetLastError();
}

hipError_t launch_advance_epoch(int64_t* epoch, hipStream_t st) {
    hipLaunchKernelGGL(advance_epoch_kernel, dim3(1), dim3(1), 0, st, epoch);
    return hipGetLastError();
}

hipError_t launch_exchange(const ExchArgs& a, int grid, hipStream_t st) {
    hipLaunchKernelGGL(exchange_kernel, dim3(grid), dim3(256), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(commit_exchange_kernel, dim3(1), dim3(1), 0, st, a.ctr, a.sp_cap);
    return hipGetLastError();
}

hipError_t launch_gather(const double* V, const int64_t* perm, double* dst, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(gather_kernel, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, V, perm, dst, n);
    return hipGetLastError();
}

hipError_t launch_scatter(double* V, const int64_t* perm, const double* src, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(scatter_kernel, dim3(unsigned((n + 255) / 256)), dim3(256), 0, st, V, perm, src, n);
    return hipGetLastError();
}

}  // namespace arbmi
