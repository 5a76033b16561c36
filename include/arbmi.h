/*
 * arbmi.h -- C ABI of the MI355X multi-compartment cell stepper.
 *
 * The library advances networks of morphologically detailed cells by the
 * scheme of the Arbor paper (arXiv:1901.07454), Section II "Model": each
 * cell is a branching cable discretised into vertex-centred control volumes
 * (eq. 2a); a time step computes membrane currents at V(t), solves the
 * implicit-Euler system for V(t+dt) with the Hines (tree Thomas) algorithm,
 * then integrates channel and synapse states with the new voltage; spikes are
 * threshold crossings on the soma and reach their targets through
 * (source, destination, synapse, delay, weight) connections, exchanged once
 * per epoch no longer than the minimum delay (Sec. II; Sec. IV-A).
 *
 * Conventions for every call
 *   - Units: V mV, t ms (steps of dt), length and diameter um, area um^2,
 *     capacitance pF, conductance nS, current pA at the interface of the
 *     numerics; densities in S/cm^2 and uF/cm^2, synaptic weights in uS,
 *     clamp amplitudes in nA (positive depolarises).
 *   - All arithmetic is IEEE FP64.
 *   - Inputs are borrowed for the duration of the call only; the library
 *     copies what it keeps.  Output buffers are owned by the caller.  A
 *     pointer documented as "device" must be a device address on the sim's
 *     GPU; "host" pointers are ordinary host memory.
 *   - Device memory is obtained through arb_params.alloc (or hipMalloc when
 *     it is NULL) and returned through arb_params.free at arb_free.
 *   - Work is enqueued on arb_params.hip_stream (NULL = the null stream).
 *     arb_step returns once its work is enqueued; every arb_get_* call
 *     synchronises that stream first.
 *   - Every call returns ARB_OK (0) or a negative ARB_E* code and never
 *     aborts or throws.  arb_last_error() gives a text for the last failure
 *     on the calling thread.  One sim must not be used from two threads at
 *     once.
 *   - User CV numbering: cells in order; within a cell the soma CV first,
 *     then each branch's CVs from proximal to distal, branches in the order
 *     given.  Voltages and traces are reported in this order even though the
 *     library stores CVs in its own packed order.
 */
#ifndef ARBMI_H
#define ARBMI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    ARB_OK = 0,
    ARB_EINVAL = -1,    /* bad model or argument (topology, sizes, ranges, NaN) */
    ARB_ENOMEM = -2,    /* the allocator returned NULL */
    ARB_EHIP = -3,      /* a HIP runtime call failed; text in arb_last_error */
    ARB_ESTATE = -4,    /* call out of order (e.g. backward before forward) */
    ARB_EOVERFLOW = -5  /* a fixed-capacity buffer (spikes, events) overflowed */
};

#define ARB_MECH_HH 1u  /* Hodgkin-Huxley Na, K and leak channels */
#define ARB_MECH_PAS 2u /* passive leak g_pas (V - e_pas) */

typedef struct arb_sim_ *arb_sim;

/* One unbranched dendritic section (Sec. II: the cell is a branching
 * one-dimensional cable).  Discretised into n_cv control volumes of equal
 * length; node k (k = 1..n_cv) sits at k*length/n_cv from the proximal end,
 * whose node is the parent's last node (or the soma). */
typedef struct {
    int32_t parent;        /* parent branch index within the cell, -1 = soma; must be < own index */
    int32_t n_cv;          /* >= 1 */
    double length_um;      /* > 0 */
    double diam_um;        /* > 0 */
    uint32_t mech;         /* ARB_MECH_HH | ARB_MECH_PAS */
    uint32_t reserved;
    double gbar_na, gbar_k, gl_hh; /* hh densities, S/cm^2 */
    double g_pas, e_pas;           /* pas density S/cm^2, reversal mV */
} arb_branch;

/* One cell: an isopotential soma node plus branches[branch_begin ..
 * branch_begin + n_branch) of the flat branch array, in topological order. */
typedef struct {
    int64_t branch_begin;
    int32_t n_branch;      /* >= 0 */
    uint32_t soma_mech;
    double soma_area_um2;  /* > 0 */
    double soma_gbar_na, soma_gbar_k, soma_gl_hh, soma_g_pas, soma_e_pas;
    double cm_uF_cm2;      /* > 0 */
    double Ra_ohm_cm;      /* > 0 */
} arb_cell;

/* Exponential synapse g' = -g/tau, current g (V - e_rev) (point source of
 * eq. 1a/2a).  branch = -1 places it on the soma (cv must be 0). */
typedef struct {
    int32_t cell, branch, cv; /* cv: 0-based CV along the branch, proximal first */
    int32_t reserved;
    double tau_ms;            /* > 0 */
    double e_rev_mV;
} arb_synapse;

/* Connection tuple (source, destination, synapse, delay, weight) (Sec. II).
 * syn is an index into the synapse array and must lie on cell dst; src is a
 * cell, or in dry-run mode any gid of the R ranks (arb_params). */
typedef struct {
    uint32_t src, dst, syn;
    int32_t delay_steps;      /* >= 1 */
    double w_uS;
} arb_connection;

/* External input event: at the start of step `step`, g[syn] += 1000 w. */
typedef struct {
    uint32_t syn;
    int32_t reserved;
    int64_t step;             /* >= 0 */
    double w_uS;
} arb_event;

/* Current clamp, active for step_on <= n < step_off. */
typedef struct {
    int32_t cell, branch, cv, reserved;
    int64_t step_on, step_off;
    double amp_nA;
} arb_iclamp;

/* A generated density mechanism on one region of a cell: the soma or one
 * branch (the role of the paper's NMODL mechanisms, Sec. III-C
 * "Mechanisms": each is described once in the description language and
 * compiled into the kernels).  Its current density, with the instance's
 * parameters and states, applies to the membrane area of every CV that lies
 * on the region (as the built-in densities do, eq. 2a).  Several entries may
 * name one region; their currents add. */
typedef struct {
    int32_t cell;
    int32_t branch;           /* branch index within the cell, -1 = the soma */
    int32_t mech;             /* index in the catalogue (arb_mechanism_info) */
    int32_t n_param;          /* param[0 .. n_param) given (in the mechanism's order);
                                 the rest take their defaults */
    double param[8];
} arb_density;

/* One mechanism of the generated catalogue. */
typedef struct {
    char name[32];
    int32_t n_params, n_states;
    char param_names[8][16];
    double defaults[8];
} arb_mech_info;

typedef struct {
    double dt_ms;             /* > 0 */
    double threshold_mV;      /* soma spike threshold (upward crossing) */
    double v_init_mV;         /* initial V; gates start at steady state, g = 0 */
    int32_t epoch_steps;      /* 0 = the minimum connection delay (at most 16384 in a
                                 network); must not exceed either */
    int32_t flags;            /* ARB_FLAG_* */
    void *hip_stream;         /* hipStream_t, NULL = null stream */
    void *(*alloc)(size_t bytes, void *ctx); /* device allocator, NULL = hipMalloc */
    void (*free)(void *ptr, void *ctx);
    void *alloc_ctx;
    int64_t spike_capacity;   /* spikes kept between arb_get_spikes calls; 0 = default */
    int64_t event_capacity;   /* network events per (cell pack, epoch); 0 = 4 x the busiest
                                 pack's incoming connections */
    int32_t block_threads;    /* threads per cell pack; 0 = autotuned */
    int32_t coef_mode;        /* 0 = autotuned, 1 = per-CV coefficients in LDS, 2 = streamed,
                                 3 = held in registers (by default for branches of <= 16 CVs;
                                 on request longer branches are cut into chains of 8-CV
                                 segments; with ARB_FLAG_GRADIENTS the packs must also fit
                                 the register-resident adjoint kernel) */
    int32_t cells_per_pack;   /* most cells one workgroup advances; 0 = autotuned */
    int32_t dry_run_ranks;    /* dry-run mode (Sec. V-E): 0 or 1 = off; R > 1: the model's cells
                                 are rank 0 of R identical ranks, connection sources may be any
                                 gid in [0, R n_cells), and the spikes of gid g on another rank
                                 are proxies: those of local cell g mod n_cells.  Each epoch's
                                 exchange then indexes R times the local spikes.  At most 2^20
                                 ranks and R n_cells < 2^31. */
    int32_t reserved0;
    const arb_density *densities; /* generated density mechanisms (read during the build only);
                                     they run in the register-resident layout (coef_mode 0 or 3,
                                     ARB_FLAG_AUTOTUNE ignored) and not with ARB_FLAG_GRADIENTS,
                                     the variable time step or state held in HBM */
    int64_t n_densities;
} arb_params;

#define ARB_FLAG_TIME_KERNELS 1 /* record HIP events around every step kernel */
#define ARB_FLAG_GRADIENTS 2    /* size cell packs so the adjoint kernel fits (use with arb_grad_*) */
#define ARB_FLAG_GRAPH 4        /* replay whole epochs from a captured HIP graph */
#define ARB_FLAG_AUTOTUNE 8     /* time candidate launch shapes on a sample of the cells at build;
                                   cached by model shape and device in the file named by the
                                   environment variable ARB_AUTOTUNE_CACHE, if set */

typedef struct {
    uint32_t gid;
    int32_t reserved;
    int64_t step;             /* index of the step whose end value crossed: V^{step-1} < thr <= V^{step} */
    double t_ms;              /* linearly interpolated crossing time (reported only) */
} arb_spike;

typedef struct {
    int32_t n_cells;
    int32_t n_packs;          /* workgroups of the step kernel */
    int64_t n_cv;             /* user CVs */
    int64_t n_slots;          /* packed CV slots incl. padding */
    int64_t n_hh, n_syn, n_conn;
    int64_t step;             /* steps completed */
    int32_t epoch_steps;
    int32_t block_threads;
    int32_t coef_mode;        /* 1 = LDS, 2 = streamed, 3 = registers */
    int32_t lds_bytes;        /* dynamic LDS per workgroup */
    int64_t device_bytes;     /* device memory held by the sim */
    int64_t bytes_per_step;   /* algorithmic HBM bytes one step must move (SoA model) */
    int32_t reg_slots;        /* coef_mode 3: branches per thread held in registers */
    int32_t reg_len;          /* coef_mode 3: CVs per branch held in registers */
    int32_t syn_hbm;          /* coef_mode 3: 1 if some workgroup keeps state in HBM: streams its
                                 synapse state every step (too many synapses for LDS), or reads
                                 its hh conductances from HBM (a cell too large for LDS
                                 otherwise); else 0 */
    int32_t n_classes;        /* launches per step kernel call: classes of workgroups that need
                                 different kernel variants or LDS, run concurrently (0 in
                                 arb_plan_layout) */
} arb_info;

/* Build a simulation from a fully enumerated model (Sec. III-A: cells,
 * their connections; Sec. II: mechanisms, synapses, injections).  Validates
 * everything on the host first (ARB_EINVAL with a message naming the bad
 * item), discretises each cell, packs cells into workgroups, uploads.
 * *out receives the new sim, or NULL on failure. */
int arb_build_cells(const arb_cell *cells, int32_t n_cells, const arb_branch *branches,
                    int64_t n_branches, const arb_synapse *syn, int64_t n_syn,
                    const arb_connection *conn, int64_t n_conn, const arb_event *ev,
                    int64_t n_ev, const arb_iclamp *stim, int32_t n_stim,
                    const arb_params *p, arb_sim *out);

/* Build a simulation that shortens steps at event times (Sec. II: the
 * step is cut so that every event falls at the beginning of a step, with
 * each cell keeping its own time).  The model is as for arb_build_cells
 * with continuous times in place of step indices: delay_ms[k] (>= dt) is the
 * delay of conn[k] (its delay_steps is validated but not used) and t_ms[k]
 * (in [0, 2^31 dt)) the time of ev[k] (its step is not used); either array
 * may be NULL when its count is 0.  A cell in [k dt, (k+1) dt) takes every
 * event due at or before its time (network events first), then steps to
 * (k+1) dt or to its next event's time if that comes first; a step from
 * k dt to (k+1) dt has length dt exactly.  A spike's time is its threshold
 * crossing interpolated within its step, and its events arrive at that time
 * plus the delay.  Epochs are K grid steps with K dt at most the minimum
 * delay (epoch_steps = 0: the largest such K), so arb_step(n) still advances
 * every cell by n steps of the grid.  arb_get_spikes reports step = -1 and
 * the spike time, sorted by (time, gid).
 * Runs one cell per workgroup in the register-resident layout
 * (coef_mode and cells_per_pack are set by the library, block_threads is
 * honoured if given, ARB_FLAG_AUTOTUNE is ignored).  ARB_EINVAL for current
 * clamps, ARB_FLAG_GRADIENTS, dry_run_ranks > 1, a cell whose synapses do
 * not fit LDS, and for the state calls (arb_get_state, arb_set_state) and
 * arb_grad_forward on the sim. */
int arb_build_cells_timed(const arb_cell *cells, int32_t n_cells, const arb_branch *branches,
                          int64_t n_branches, const arb_synapse *syn, int64_t n_syn,
                          const arb_connection *conn, const double *delay_ms, int64_t n_conn,
                          const arb_event *ev, const double *t_ms, int64_t n_ev,
                          const arb_params *p, arb_sim *out);

/* Steps taken by all cells since the build into *n_out: with the variable
 * time step, every cell's full and shortened steps (Sec. II); otherwise the
 * completed steps times the cell count.  Synchronises the sim's stream. */
int arb_get_step_count(arb_sim s, int64_t *n_out);

/* The generated mechanism catalogue: the number of mechanisms, and the
 * name, parameters (names, defaults) and state count of mechanism id
 * (0 .. count - 1).  ARB_EINVAL for an id out of range. */
int arb_mechanism_count(void);
int arb_mechanism_info(int32_t id, arb_mech_info *out);

/* Instances of each generated mechanism in the sim (Sec. III-C: a density
 * mechanism acts on every CV that its region covers, one instance per CV
 * and density entry) into counts[id], id = 0 .. n - 1 (zero past the
 * catalogue).  counts is host memory owned by the caller; ARB_EINVAL for a
 * null argument or n < arb_mechanism_count(). */
int arb_get_mechanism_instances(arb_sim s, int64_t *counts, int32_t n);

/* Advance every cell by n_steps steps of dt (Sec. II operator splitting:
 * events due at the step start, currents at V(t), implicit Euler + Hines for
 * V(t+dt), states with the new V, threshold test; spike exchange at each
 * epoch end, Sec. IV-A).  Asynchronous: errors returned here are those of the
 * host (arguments, launches); on such a failure the sim is left at the last
 * completed epoch.  A spike or event buffer that fills during the steps is
 * flagged on the device (the writes past it are dropped, never made out of
 * bounds), and arb_sync and arb_get_spikes report the flag as ARB_EOVERFLOW;
 * it stays set for the life of the sim. */
int arb_step(arb_sim s, int64_t n_steps);

/* Copy all n_cv voltages V_i (the discretised voltages of eq. 2a, one per
 * control volume) in user CV order into dst (n >= n_cv doubles), a device
 * pointer if dst_on_device, else host.  The paper validates its models by
 * comparing the voltage traces of individual cells (Sec. V-A, "Models").
 * A host dst is staged through a device buffer the sim allocates on the
 * first such call and keeps until arb_free. */
int arb_get_voltages(arb_sim s, double *dst, int64_t n, int dst_on_device);

/* arb_get_voltages into host memory without allocating: for callers that
 * cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid it).  Same output as arb_get_voltages with a
 * host dst (n >= n_cv doubles, user CV order), staged through a fixed 64 MiB
 * array of static device memory (8,388,608 doubles) that every GPU the
 * library runs on holds until the process ends.  ARB_EINVAL if the model has
 * more CVs than that (the call then touches nothing).  All sims on one GPU
 * share the array: calls that overlap on one GPU race and must not be made. */
int arb_get_voltages_noalloc(arb_sim s, double *dst, int64_t n);

/* Drain the spikes recorded since the last call into host dst, sorted by
 * (step, gid).  A spike is an upward crossing of the fixed threshold by the
 * soma voltage (Sec. II); spike trains are the second output the paper
 * validates its models by (Sec. V-A, "Models").  *n_out = number written.  ARB_EOVERFLOW if cap was too small
 * (nothing is drained then, *n_out = 0), or if a spike or event buffer has
 * overflowed (the kept spikes are still written and counted in *n_out). */
int arb_get_spikes(arb_sim s, arb_spike *dst, int64_t cap, int64_t *n_out);

/* Record V of the given user CVs after every step from now on, for up to
 * max_steps steps (the voltage traces of Sec. V-A, "Models").  Replaces
 * earlier probes; the previous probe table and trace buffer are released. */
int arb_set_probes(arb_sim s, const int64_t *cv, int32_t n, int64_t max_steps);

/* Copy the recorded voltage trace (Sec. V-A, "Models"), layout
 * [probe][step], into dst (n_probe * cap doubles, device or host) and
 * restart recording.  *n_steps_out = steps
 * recorded. */
int arb_get_trace(arb_sim s, double *dst, int64_t cap, int dst_on_device, int64_t *n_steps_out);

/* Replace per-region channel densities theta[cell][region][3] =
 * (gbar_na, gbar_k, g_pas), region 0 = soma, 1 + b = branch b (host array of
 * n = 3 * (n_cells + n_branches) doubles).  These are the areal conductances
 * g_k of the channel terms S_i g_k (V_i - e_k) in eq. 2a.  Takes effect at
 * the next step. */
int arb_set_params(arb_sim s, const double *theta, int64_t n);

/* Gradient support (discrete adjoint of the step).  An addition beyond the
 * paper, which computes no gradients: the adjoint differentiates exactly the
 * operator-split implicit-Euler step of Sec. II.  Forward: run n_steps
 * recording the soma voltage of every cell after each step into trace_dev
 * (device, [cell][step]), storing a state checkpoint every ckpt_every
 * steps; input events are recorded and treated as fixed in the backward.
 * Probes set with arb_set_probes are suspended for these steps and resume
 * afterwards, their recording restarted at the step the forward ends at. */
int arb_grad_forward(arb_sim s, int64_t n_steps, int32_t ckpt_every, double *trace_dev);

/* Backward: given dL/dtrace (device, [cell][step]), write dL/dtheta (device,
 * [cell][region][3], layout of arb_set_params).  ARB_ESTATE without a prior
 * arb_grad_forward.  Leaves the sim's state at the end of the forward. */
int arb_grad_backward(arb_sim s, const double *dL_dtrace_dev, double *dL_dtheta_dev);

/* Checkpoint: serialise / restore the dynamic state (an addition beyond the
 * paper, which describes no checkpointing: step, V, gates,
 * synaptic conductances, pending events, event cursors, spike buffer and
 * history).  With blob NULL, arb_get_state writes only the size into *n_out.
 * arb_set_state takes a blob of the same model (ARB_EINVAL otherwise, or if
 * any cursor, offset, synapse index or gid in it is out of range; the sim is
 * then unchanged). */
int arb_get_state(arb_sim s, void *blob, int64_t cap, int64_t *n_out);
int arb_set_state(arb_sim s, const void *blob, int64_t n);

/* Sizes and the chosen launch configuration. */
int arb_get_info(arb_sim s, arb_info *info);

/* Plan without a device: validate and lower the model exactly as
 * arb_build_cells would with these parameters (launch parameters 0 are
 * planned as if on an MI355X: 256 CUs, 160 KiB LDS), check the packed
 * layout's invariants (every CV in one slot; children eliminated before their
 * parents; each thread's register slot used by one branch), and report sizes
 * in info (step = 0, device_bytes = 0).  No device memory is touched.
 * ARB_EINVAL on a bad model or a violated invariant (message names it). */
int arb_plan_layout(const arb_cell *cells, int32_t n_cells, const arb_branch *branches,
                    int64_t n_branches, const arb_synapse *syn, int64_t n_syn,
                    const arb_connection *conn, int64_t n_conn, const arb_event *ev,
                    int64_t n_ev, const arb_iclamp *stim, int32_t n_stim,
                    const arb_params *p, arb_info *info);

/* Step-kernel timing (ARB_FLAG_TIME_KERNELS): total ms and number of
 * launches since the last call; synchronises the stream. */
int arb_get_kernel_time(arb_sim s, double *ms_total, int64_t *n_launches);

/* Wait for all enqueued work of the sim.  ARB_EOVERFLOW if a spike or event
 * buffer has overflowed (arb_step). */
int arb_sync(arb_sim s);

/* Release everything the sim holds.  NULL is accepted. */
int arb_free(arb_sim s);

/* Text of the last failure on the calling thread ("" if none). */
const char *arb_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* ARBMI_H */
