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

#include <algorithm>
#include <climits>

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

    // external-event cursor in thread 0's registers, with the next step cached
    int64_t step0 = a.step0;
    if (a.epoch_ptr) step0 = *a.epoch_ptr * a.nsteps;
    const int64_t estart = step0 - step0 % a.epoch_steps;  // the epoch's first step
    const uint32_t* eoff = a.bk_off ? a.bk_off + int64_t(p) * (a.epoch_steps + 1) : nullptr;
    const int32_t* eq = a.bk_q + int64_t(p) * a.bk_cap;
    const double* ew = a.bk_w + int64_t(p) * a.bk_cap;
    int64_t xcur = 0;
    int64_t xstep = INT64_MAX;
    int32_t eb = INT32_MAX;  // the next step of the epoch with network events
    if (tid == 0) {
        xcur = a.pk_xcur[p];
        if (xcur < pk.xe1) xstep = a.xe_step[xcur];
        if (eoff) eb = int32_t(a.bk_nxt[int64_t(p) * (a.epoch_steps + 1) + (step0 - estart)]);
    }
    const int soma = (tid < pk.ncell) ? a.pc_soma[pk.cell0 + tid] : -1;
    double vold = 0.0;
    __syncthreads();

    for (int s = 0; s < a.nsteps; ++s) {
        const int64_t n = step0 + s;

        // A: events due at the start of step n (network, then external)
        if (tid == 0) {
            const int32_t b = int32_t(n - estart);
            if (b == eb) {
                const uint32_t i0 = eoff[b], i1 = eoff[b + 1];
                eb = int32_t(a.bk_nxt[int64_t(p) * (a.epoch_steps + 1) + b + 1]);
                for (uint32_t i = i0; i < i1; ++i) sg[eq[i]] += ew[i];
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
    if (tid == 0) a.pk_xcur[p] = xcur;
}

// ---------------------------------------------------------------------------
// Spike exchange between epochs.  An event reaches its synapse no earlier
// than the minimum delay after the spike (Sec. II), and an epoch is no
// longer than that, so the events of epoch e come only from spikes of
// earlier epochs.  At each epoch end the epoch's spikes are copied into a
// ring of per-epoch history slots covering the longest delay; at each epoch
// start the history is indexed by source gid and every pack pulls its
// incoming connections (ranks in order) against the index, writing its
// bucket of the epoch already in (step, rank) order.

// The epoch's spikes [sp_exch, sp_count) into history slot epoch % n_hist,
// over any number of workgroups (every block reads the counters, which only
// collect_finish_kernel moves, after this kernel).
__global__ void __launch_bounds__(256) collect_copy_kernel(const Counters* ctr, const uint32_t* sp_gid,
                                                           const int64_t* sp_step, uint32_t sp_cap, uint32_t* h_gid,
                                                           int64_t* h_step, uint32_t h_cap, int32_t n_hist,
                                                           int64_t epoch, const int64_t* epoch_ptr) {
    const int64_t e = epoch_ptr ? *epoch_ptr : epoch;
    const int64_t slot = e % n_hist;
    const uint32_t b = ctr->sp_exch;
    const uint32_t end = ctr->sp_count < sp_cap ? ctr->sp_count : sp_cap;
    const uint32_t n = end > b ? end - b : 0u;
    const uint32_t m = n < h_cap ? n : h_cap;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) {
        h_gid[slot * h_cap + i] = sp_gid[b + i];
        h_step[slot * h_cap + i] = sp_step[b + i];
    }
}

// The slot's count, the overflow flag, and the exchanged mark.
__global__ void collect_finish_kernel(Counters* ctr, uint32_t sp_cap, uint32_t* h_cnt, uint32_t h_cap,
                                      int32_t n_hist, int64_t epoch, const int64_t* epoch_ptr) {
    const int64_t e = epoch_ptr ? *epoch_ptr : epoch;
    const uint32_t b = ctr->sp_exch;
    const uint32_t end = ctr->sp_count < sp_cap ? ctr->sp_count : sp_cap;
    const uint32_t n = end > b ? end - b : 0u;
    h_cnt[e % n_hist] = n < h_cap ? n : h_cap;
    if (n > h_cap) atomicOr(&ctr->flags, kFlagEventOverflow);
    ctr->sp_exch = end;
}

// Index the history's spikes by source gid over any number of workgroups:
// count per gid, an exclusive scan of the counts into off[0, n_src] (tiles
// of kScanTile gids: scanned per tile, tile totals scanned, tile offsets
// added), then scatter the steps while counting back down, which leaves the
// counts at zero for the next epoch.  With R ranks (dry run) every local
// spike of gid g stands for R spikes, of gids g + k n_cells, k < R; the
// index holds at most sx_cap of them (in history order, spike by spike),
// and more flag an event overflow.
constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;

struct IndexArgs {
    const uint32_t* h_gid;
    const int64_t* h_step;
    const uint32_t* h_cnt;
    uint32_t h_cap;
    int32_t n_hist;
    int32_t ranks;      // R
    int32_t n_cells;    // local cells
    int64_t n_src;      // R n_cells
    int64_t sx_cap;
    int32_t* cnt;       // [n_src]
    int64_t* off;       // [n_src + 1]
    int64_t* tile_sum;  // [tiles]
    int64_t* sx_step;   // [sx_cap]
    Counters* ctr;
};

__device__ __forceinline__ int64_t history_spikes(const IndexArgs& a) {
    int64_t n = 0;
    for (int32_t h = 0; h < a.n_hist; ++h) n += a.h_cnt[h];
    return n;
}

// f(gid, step) for every indexed proxy spike, grid-stride, in history order
template <class Fn>
__device__ __forceinline__ void for_each_proxy(const IndexArgs& a, Fn fn) {
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    int64_t base = 0;  // proxies of the earlier history slots
    for (int32_t h = 0; h < a.n_hist && base < a.sx_cap; ++h) {
        const int64_t e_h = int64_t(a.h_cnt[h]) * a.ranks;
        const int64_t lim = (base + e_h <= a.sx_cap) ? e_h : a.sx_cap - base;
        for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < lim; i += stride) {
            const int64_t sp = i / a.ranks, k = i - sp * a.ranks;
            const int64_t at = int64_t(h) * a.h_cap + sp;
            fn(int64_t(a.h_gid[at]) + k * a.n_cells, a.h_step[at]);
        }
        base += e_h;
    }
}

__global__ void __launch_bounds__(256) index_count_kernel(IndexArgs a) {
    const int64_t n = history_spikes(a);
    if (n == 0) return;
    if (blockIdx.x == 0 && threadIdx.x == 0 && n * a.ranks > a.sx_cap) atomicOr(&a.ctr->flags, kFlagEventOverflow);
    for_each_proxy(a, [&](int64_t g, int64_t) { atomicAdd(&a.cnt[g], 1); });
}

// exclusive scan of v over the block (kScanThreads threads); *total gets the sum
__device__ __forceinline__ int64_t block_scan(int64_t v, int64_t* lds, int64_t* total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int64_t x = v;
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == 63) lds[wave] = x;
    __syncthreads();
    int64_t before = 0, all = 0;
    for (int w = 0; w < kScanThreads / 64; ++w) {
        before += (w < wave) ? lds[w] : 0;
        all += lds[w];
    }
    __syncthreads();
    *total = all;
    return before + x - v;
}

// per tile: off[i] = exclusive prefix of cnt within the tile; tile totals
__global__ void __launch_bounds__(kScanThreads) index_scan_tiles_kernel(IndexArgs a) {
    __shared__ int64_t lds[kScanThreads / 64];
    if (history_spikes(a) == 0) return;
    const int64_t t0 = int64_t(blockIdx.x) * kScanTile + int64_t(threadIdx.x) * kScanItems;
    int32_t c[kScanItems];
    int64_t sum = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        c[k] = (t0 + k < a.n_src) ? a.cnt[t0 + k] : 0;
        sum += c[k];
    }
    int64_t total;
    int64_t run = block_scan(sum, lds, &total);
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        if (t0 + k < a.n_src) a.off[t0 + k] = run;
        run += c[k];
    }
    if (threadIdx.x == 0) a.tile_sum[blockIdx.x] = total;
}

// one block: tile totals -> exclusive tile offsets (in place); off[n_src]
__global__ void __launch_bounds__(kScanThreads) index_scan_totals_kernel(IndexArgs a, int64_t tiles) {
    __shared__ int64_t lds[kScanThreads / 64];
    if (history_spikes(a) == 0) {
        if (threadIdx.x == 0) a.off[a.n_src] = 0;  // the pull checks the total first
        return;
    }
    int64_t carry = 0;
    for (int64_t b0 = 0; b0 < tiles; b0 += kScanThreads) {
        const int64_t i = b0 + threadIdx.x;
        const int64_t v = i < tiles ? a.tile_sum[i] : 0;
        int64_t total;
        const int64_t x = block_scan(v, lds, &total);
        if (i < tiles) a.tile_sum[i] = carry + x;
        carry += total;
    }
    if (threadIdx.x == 0) a.off[a.n_src] = carry;
}

__global__ void __launch_bounds__(kScanThreads) index_scan_add_kernel(IndexArgs a) {
    if (history_spikes(a) == 0) return;
    const int64_t add = a.tile_sum[blockIdx.x];
    const int64_t t0 = int64_t(blockIdx.x) * kScanTile;
    for (int k = threadIdx.x; k < kScanTile; k += kScanThreads)
        if (t0 + k < a.n_src) a.off[t0 + k] += add;
}

__global__ void __launch_bounds__(256) index_scatter_kernel(IndexArgs a) {
    if (history_spikes(a) == 0) return;
    for_each_proxy(a, [&](int64_t g, int64_t step) { a.sx_step[a.off[g] + atomicSub(&a.cnt[g], 1) - 1] = step; });
}

__device__ __forceinline__ int wave_min(int v) {
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
    return v;
}

// One wave per pack.  Pass 1 counts the epoch's events per step (LDS
// counters over the K steps), a scan turns the counts into each step's
// first position (stored as the bucket's step offsets), and pass 2 walks
// the connections again in rank order, 64 at a time: the chunk's events are
// placed step by step, increasing, a lane's event at its step's cursor plus
// the number of lower lanes with an event at that step, so every step's
// events are in rank order.  An event is stored as (pack-local synapse,
// weight).
__global__ void __launch_bounds__(64) pull_events_kernel(PullArgs a) {
    extern __shared__ uint32_t bins[];
    constexpr int U = 4;  // connections per lane in flight, spikes per source kept in registers
    const int p = blockIdx.x;
    const int lane = threadIdx.x;
    const int64_t e = a.epoch_ptr ? *a.epoch_ptr : a.epoch;
    const int K = a.epoch_steps;
    const int64_t lo = e * K;
    const int64_t r0 = a.in_off[p], r1 = a.in_off[p + 1];
    if (a.sx_off[a.n_src] == 0) {  // no spikes in the history: no events this epoch
        uint32_t* nxt = a.bk_nxt + int64_t(p) * (K + 1);
        for (int b = lane; b <= K; b += 64) nxt[b] = uint32_t(K);
        return;
    }
    for (int b = lane; b < K; b += 64) bins[b] = 0u;
    __syncthreads();
    // pass 1: U connections per lane at a time, their loads issued together
    for (int64_t c = r0; c < r1; c += 64 * U) {
        uint32_t src[U];
        int64_t d[U], k0[U], k1[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t r = c + u * 64 + lane;
            src[u] = r < r1 ? a.cr_src[r] : 0u;
            d[u] = r < r1 ? a.cr_delay[r] : 0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const bool ok = c + u * 64 + lane < r1;
            k0[u] = ok ? a.sx_off[src[u]] : 0;
            k1[u] = ok ? a.sx_off[src[u] + 1] : 0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            for (int64_t k = k0[u]; k < k1[u]; ++k) {
                const int64_t b = a.sx_step[k] + d[u] - lo;
                if (b >= 0 && b < K) atomicAdd(&bins[b], 1u);
            }
    }
    __syncthreads();
    uint32_t run = 0;
    for (int b0 = 0; b0 < K; b0 += 64) {
        const int b = b0 + lane;
        const uint32_t c = b < K ? bins[b] : 0u;
        uint32_t x = c;
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(x, o);
            if (lane >= o) x += y;
        }
        if (b < K) bins[b] = run + x - c;
        run += __shfl(x, 63);
    }
    const uint32_t total = run;
    __syncthreads();
    const uint32_t cap = uint32_t(a.bk_cap);
    uint32_t* off = a.bk_off + int64_t(p) * (K + 1);
    for (int b = lane; b < K; b += 64) off[b] = bins[b] < cap ? bins[b] : cap;
    if (lane == 0) off[K] = total < cap ? total : cap;
    // for each step, the first step at or after it with events (K if none):
    // a suffix minimum over 64 steps at a time, from the last
    {
        uint32_t* nxt = a.bk_nxt + int64_t(p) * (K + 1);
        int later = K;
        for (int b0 = ((K - 1) / 64) * 64; b0 >= 0; b0 -= 64) {
            const int b = b0 + lane;
            int x = K;
            if (b < K) {
                const uint32_t s0 = bins[b] < cap ? bins[b] : cap;
                const uint32_t e1 = b + 1 < K ? bins[b + 1] : total;
                if ((e1 < cap ? e1 : cap) > s0) x = b;
            }
            for (int o = 1; o < 64; o <<= 1) {
                const int y = __shfl_down(x, o);
                if (lane + o < 64) x = min(x, y);
            }
            x = min(x, later);
            if (b < K) nxt[b] = uint32_t(x);
            later = __shfl(x, 0);
        }
        if (lane == 0) nxt[K] = uint32_t(K);
    }
    int32_t* oq = a.bk_q + int64_t(p) * a.bk_cap;
    double* ow = a.bk_w + int64_t(p) * a.bk_cap;
    const uint64_t below = (uint64_t(1) << lane) - 1u;
    // pass 2: 64 connections at a time, this lane's event steps (the source's
    // spikes in the window, up to U of them in registers, more re-read).
    // The loads run ahead of the placement: a chunk's source and delay two
    // chunks early, its source's spike range one chunk early, so a chunk
    // waits for one round of loads (its spike steps, and its synapse and
    // weight if the source fired). Loads complete in issue order, so each
    // chunk issues its own loads before those it issues for later chunks.
    int64_t d_c = 0, k0_c = 0, k1_c = 0;  // the chunk about to run
    uint32_t src_n = 0u;                  // the chunk after it
    int64_t d_n = 0;
    {
        const int64_t r = r0 + lane;
        if (r < r1) {
            const uint32_t src = a.cr_src[r];
            d_c = a.cr_delay[r];
            k0_c = a.sx_off[src];
            k1_c = a.sx_off[src + 1];
        }
        if (r + 64 < r1) {
            src_n = a.cr_src[r + 64];
            d_n = a.cr_delay[r + 64];
        }
    }
    for (int64_t c0 = r0; c0 < r1; c0 += 64) {
        const int64_t r = c0 + lane;
        const int64_t d = d_c, k0 = k0_c, k1 = k1_c;  // k0 = k1 = 0 past r1
        int32_t q = 0;
        double w = 0.0;
        if (k1 > k0) {
            q = a.cr_syn[r];
            w = a.cr_w[r];
        }
        int64_t st[U];
#pragma unroll
        for (int u = 0; u < U; ++u) st[u] = k0 + u < k1 ? a.sx_step[k0 + u] : 0;
        // the next chunk's spike ranges, the chunk after's sources and delays
        k0_c = 0;
        k1_c = 0;
        d_c = d_n;
        if (r + 64 < r1) {
            k0_c = a.sx_off[src_n];
            k1_c = a.sx_off[src_n + 1];
        }
        src_n = 0u;
        d_n = 0;
        if (r + 128 < r1) {
            src_n = a.cr_src[r + 128];
            d_n = a.cr_delay[r + 128];
        }
        int bs[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            bs[u] = INT_MAX;
            if (k0 + u < k1) {
                const int64_t b = st[u] + d - lo;
                if (b >= 0 && b < K) bs[u] = int(b);
            }
        }
        const bool more = k1 - k0 > U;
        // fast path, when no lane has more than one event in the epoch (a
        // volley): sort the chunk's (step, lane) keys across the wave
        // (bitonic network over the lanes); an event's place among its
        // step's events is its distance from the start of its step's run,
        // which keeps lane order, as the general path below does
        int nev = more ? 2 : 0, one = K;
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (bs[u] != INT_MAX) {
                ++nev;
                one = bs[u];
            }
        if (__all(nev <= 1)) {
            uint32_t key = (uint32_t(one) << 6) | uint32_t(lane);
            for (int k = 2; k <= 64; k <<= 1)
                for (int j = k >> 1; j > 0; j >>= 1) {
                    const uint32_t other = __shfl_xor(key, j);
                    const bool low = (lane & j) == 0, up = (lane & k) == 0;
                    key = (low == up) ? min(key, other) : max(key, other);
                }
            const int b = int(key >> 6), from = int(key & 63u);
            const int32_t qq = __shfl(q, from);
            const double ww = __shfl(w, from);
            const int prev = __shfl_up(b, 1), next = __shfl_down(b, 1);  // every lane shuffles
            const bool start = lane == 0 || prev != b;
            const bool end = lane == 63 || next != b;
            const uint64_t starts = __ballot(start) & ((uint64_t(2) << lane) - 1u);
            const uint32_t rank = uint32_t(lane - (63 - __clzll(starts)));
            const uint32_t base = (b < K) ? bins[b] : 0u;
            if (b < K) {
                const uint32_t pos = base + rank;
                if (pos < cap) {
                    oq[pos] = qq;
                    ow[pos] = ww;
                }
            }
            __builtin_amdgcn_wave_barrier();
            if (b < K && end) bins[b] = base + rank + 1u;
            __builtin_amdgcn_wave_barrier();
            continue;
        }
        int last = -1;
        for (;;) {
            int mine = INT_MAX;  // this lane's first event step after `last`
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (bs[u] > last && bs[u] < mine) mine = bs[u];
            if (more)
                for (int64_t k = k0 + U; k < k1; ++k) {
                    const int64_t b = a.sx_step[k] + d - lo;
                    if (b > last && b < K && b < mine) mine = int(b);
                }
            const int B = wave_min(mine);
            if (B == INT_MAX) break;
            const uint64_t mask = __ballot(mine == B);
            const uint32_t base = bins[B];
            if (mine == B) {
                const uint32_t pos = base + uint32_t(__popcll(mask & below));
                if (pos < cap) {
                    oq[pos] = q;
                    ow[pos] = w;
                }
            }
            // one wave: its LDS operations take effect in issue order, so a
            // wave barrier orders the cursor's read and update without
            // waiting for the event stores
            __builtin_amdgcn_wave_barrier();
            if (lane == 0) bins[B] = base + uint32_t(__popcll(mask));
            __builtin_amdgcn_wave_barrier();
            last = B;
        }
    }
    if (lane == 0 && total > cap) atomicOr(&a.ctr->flags, kFlagEventOverflow);
}

__global__ void advance_epoch_kernel(int64_t* epoch) { *epoch += 1; }

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
                         reinterpret_cast<const void*>(&pull_events_kernel)};
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

hipError_t launch_advance_epoch(int64_t* epoch, hipStream_t st) {
    hipLaunchKernelGGL(advance_epoch_kernel, dim3(1), dim3(1), 0, st, epoch);
    return hipGetLastError();
}

hipError_t launch_collect_spikes(Counters* ctr, const uint32_t* sp_gid, const int64_t* sp_step, uint32_t sp_cap,
                                 uint32_t* h_gid, int64_t* h_step, uint32_t* h_cnt, uint32_t h_cap, int32_t n_hist,
                                 int64_t epoch, const int64_t* epoch_ptr, hipStream_t st) {
    const unsigned nb = unsigned(std::min<int64_t>(256, std::max<int64_t>(1, (int64_t(h_cap) + 255) / 256)));
    hipLaunchKernelGGL(collect_copy_kernel, dim3(nb), dim3(256), 0, st, ctr, sp_gid, sp_step, sp_cap, h_gid, h_step,
                       h_cap, n_hist, epoch, epoch_ptr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(collect_finish_kernel, dim3(1), dim3(1), 0, st, ctr, sp_cap, h_cnt, h_cap, n_hist, epoch,
                       epoch_ptr);
    return hipGetLastError();
}

int64_t index_tiles(int64_t n_src) { return (n_src + kScanTile - 1) / kScanTile; }

hipError_t launch_index_spikes(const IndexLaunch& x, hipStream_t st) {
    IndexArgs a{};
    a.h_gid = x.h_gid;
    a.h_step = x.h_step;
    a.h_cnt = x.h_cnt;
    a.h_cap = x.h_cap;
    a.n_hist = x.n_hist;
    a.ranks = x.ranks;
    a.n_cells = x.n_cells;
    a.n_src = int64_t(x.ranks) * x.n_cells;
    a.sx_cap = x.sx_cap;
    a.cnt = x.cnt;
    a.off = x.off;
    a.tile_sum = x.tile_sum;
    a.sx_step = x.sx_step;
    a.ctr = x.ctr;
    const int64_t tiles = index_tiles(a.n_src);
    // proxies per epoch: about R x the spikes of the history; enough blocks
    // for every CU, more when the dry run multiplies them
    const unsigned nb = unsigned(std::min<int64_t>(4096, std::max<int64_t>(256, int64_t(x.ranks) * 4)));
    hipLaunchKernelGGL(index_count_kernel, dim3(nb), dim3(256), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(index_scan_tiles_kernel, dim3(unsigned(tiles)), dim3(kScanThreads), 0, st, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(index_scan_totals_kernel, dim3(1), dim3(kScanThreads), 0, st, a, tiles);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(index_scan_add_kernel, dim3(unsigned(tiles)), dim3(kScanThreads), 0, st, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(index_scatter_kernel, dim3(nb), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_pull_events(const PullArgs& a, int32_t n_packs, hipStream_t st) {
    hipLaunchKernelGGL(pull_events_kernel, dim3(n_packs), dim3(64), size_t(a.epoch_steps) * 4, st, a);
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
