/*
 * oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, scalar FP64 CPU reference for the per-time-step update of
 * networks of multi-compartment cells (Arbor paper, Section II "Model").
 * Only the tests, the smoke check and the CPU-baseline leg of the benchmark
 * load it; the GPU library neither links nor calls it, and this file shares
 * no code, header, table or helper with the GPU library.
 *
 * What it follows, in the paper's order and notation:
 *   - vertex-centred finite volumes, first-order axial flux (Sec. II, eq. 2a):
 *     c_i dV_i/dt = sum_j sigma_ij (V_j - V_i) - I_inj - I_syn - S_i g_k (V_i - e_k)
 *   - operator splitting (Sec. II): currents from V(t); V(t+dt) by implicit
 *     Euler; then mechanism states integrated with the updated V.
 *   - the implicit-Euler linear system (Sec. II, unnumbered):
 *     (c_i/dt) V'_i + sum_j sigma_ij V'_i - sum_j sigma_ij V'_j = -I_i + (c_i/dt) V_i
 *   - parent-before-child numbering, solved by the extended Thomas (Hines)
 *     algorithm: leaves-to-root elimination, root-to-leaves substitution.
 *   - spikes: threshold crossing on the soma (Sec. II); connections are
 *     (source, destination, synapse, delay, weight) tuples; spikes are
 *     exchanged once per epoch of at most the minimum delay (Sec. II and
 *     Sec. IV-A "Simulation workflow"); events apply at the start of a step.
 * Readings for what the paper leaves open (node placement, soma, mixed-CV
 * mechanism areas, hh/pas/expsyn equations, threshold, injection sign, event
 * order) are the ones listed in the design notes; each is marked READING below.
 *
 * Parity pins: every function here is checked in tests against something
 * other than itself (dense LU, banded solve, closed-form cable responses,
 * charge conservation, textbook HH resting values and firing rate, exact
 * exponential decay, epoch invariance, finite differences).
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (no fast-math).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define MECH_HH 1u
#define MECH_PAS 2u

/* READING: textbook Hodgkin-Huxley reversal potentials (mV). */
#define E_NA 50.0
#define E_K (-77.0)
#define E_L (-54.3)

typedef struct {
    int64_t step;
    int32_t kind; /* 0 = network (spike-driven), 1 = external input */
    uint32_t syn;
    uint32_t src;
    int64_t seq;
    double w; /* uS */
} orc_event;

typedef struct {
    uint32_t gid;
    int64_t step;
    double t;
} orc_spike;

/* an event of the variable-step mode: continuous time (ms) */
typedef struct {
    int32_t cell;
    double t;
    int32_t kind; /* 0 = network, 1 = external input */
    uint32_t syn;
    uint32_t src;
    int64_t seq;
    double w; /* uS */
} orc_tev;

typedef struct {
    /* sizes */
    int32_t ncell;
    int64_t ncv, nreg, nsyn, ncon, nic;
    double dt, theta, v0;
    int32_t K; /* epoch length in steps */

    /* discretisation */
    int64_t *cv_begin;  /* [ncell+1] */
    int64_t *reg_begin; /* [ncell+1]; region 0 of a cell = soma, 1+b = branch b */
    int64_t *parent;    /* [ncv] global parent CV, -1 at the soma */
    double *cap;        /* [ncv] pF */
    double *sig;        /* [ncv] nS between CV and its parent (0 at soma) */
    int64_t *ct_begin;  /* [ncv+1] membrane pieces (region, area) of each CV */
    int64_t *ct_reg;
    double *ct_area; /* um^2 */
    int8_t *has_hh;  /* [ncv] */
    int64_t *lpar;   /* [ncv] parent as a cell-local index, -1 at the soma */
    double *uoff;    /* [ncv] off-diagonal entry -sigma linking a CV to its parent */

    /* regions */
    uint32_t *reg_mech;
    double *reg_gna, *reg_gk, *reg_gl, *reg_gpas, *reg_epas; /* S/cm^2, mV */
    int64_t *reg_cell;

    /* synapses */
    int64_t *syn_cv;
    double *syn_tau, *syn_e;

    /* connections, grouped by source */
    int64_t *out_begin; /* [ncell+1] */
    uint32_t *out_syn, *out_src;
    int32_t *out_delay;
    double *out_w;
    int64_t *out_id;

    /* current clamps */
    int64_t *ic_cv, *ic_on, *ic_off;
    double *ic_amp;

    /* state */
    int64_t step;
    double *V, *m, *h, *n, *g;

    /* pending events, sorted, consumed from ev_head */
    orc_event *ev;
    int64_t nev, capev, ev_head;

    /* spikes */
    orc_spike *sp;
    int64_t nsp, capsp, sp_epoch_begin;

    /* optional recording of every delivered event (for the adjoint) */
    int record_events;
    orc_event *rec;
    int64_t nrec, caprec;

    /* scratch */
    double *d, *rhs, *I;

    /* variable-step mode (orc_set_varstep) */
    int varstep;
    int64_t K_ep;          /* epoch length (grid steps) */
    int64_t k_now;         /* grid point every cell has reached */
    double *tcell;         /* [ncell] each cell's time */
    int64_t *kcell;        /* [ncell] its grid interval: k dt <= t < (k+1) dt */
    double *out_delay_ms;  /* per connection, out_* order */
    int32_t *syn_cell;     /* [nsyn] */
    int64_t *csyn_begin, *csyn; /* synapses of each cell */
    orc_tev *tev;          /* pending events */
    int64_t ntev, captev;
    int64_t *tev_begin, *tev_end, *tev_head; /* [ncell] this epoch's events of each cell */
    int64_t nvsteps;       /* steps taken (all cells) */

    /* further density mechanisms (orc_set_densities): instances per CV */
    int64_t ngen;
    int64_t *gen_begin;    /* [ncv+1] instances of each CV */
    int32_t *gen_mech;     /* ORC_GEN_* */
    double *gen_w;         /* 10 x area (um^2): S/cm^2 -> nS */
    double *gen_p;         /* [ngen][8] parameters */
    double *gen_s;         /* [ngen][4] states */
} orc;

/* ------------------------------------------------------------------------ */
/* hh rate functions (READING: textbook HH at 6.3 C, q10 factor 1)           */

/* x / (exp(x) - 1), with its removable singularity at x = 0 */
static double exprelr(double x) {
    if (1.0 + x == 1.0) return 1.0;
    return x / expm1(x);
}

/* d/dx exprelr(x) */
static double exprelr_dx(double x) {
    if (fabs(x) < 1e-4) return -0.5 + x / 6.0 - x * x * x / 180.0;
    double em = expm1(x);
    return (em - x * (em + 1.0)) / (em * em);
}

/* rates r[0..5] = alpha_m, beta_m, alpha_h, beta_h, alpha_n, beta_n (1/ms) */
void orc_hh_rates(double v, double *r) {
    r[0] = exprelr(-(v + 40.0) / 10.0);
    r[1] = 4.0 * exp(-(v + 65.0) / 18.0);
    r[2] = 0.07 * exp(-(v + 65.0) / 20.0);
    r[3] = 1.0 / (exp(-(v + 35.0) / 10.0) + 1.0);
    r[4] = 0.1 * exprelr(-(v + 55.0) / 10.0);
    r[5] = 0.125 * exp(-(v + 65.0) / 80.0);
}

/* derivatives of the six rates with respect to v */
void orc_hh_rates_dv(double v, double *r) {
    r[0] = -0.1 * exprelr_dx(-(v + 40.0) / 10.0);
    r[1] = -4.0 / 18.0 * exp(-(v + 65.0) / 18.0);
    r[2] = -0.07 / 20.0 * exp(-(v + 65.0) / 20.0);
    double u = exp(-(v + 35.0) / 10.0);
    r[3] = 0.1 * u / ((1.0 + u) * (1.0 + u));
    r[4] = -0.01 * exprelr_dx(-(v + 55.0) / 10.0);
    r[5] = -0.125 / 80.0 * exp(-(v + 65.0) / 80.0);
}

/* ------------------------------------------------------------------------ */
/* Hines solve (Sec. II): A x = b with A symmetric, diagonal d, off-diagonal
 * entry u[i] linking CV i to parent[i] < i.  Elimination from the highest
 * index down to the root, then substitution upwards.  d and b are
 * overwritten; the solution is left in b. */
void orc_hines_solve(int64_t n, const int64_t *parent, double *d, const double *u, double *b) {
    for (int64_t i = n - 1; i >= 0; --i) {
        int64_t p = parent[i];
        if (p < 0) continue;
        double f = u[i] / d[i];
        d[p] -= f * u[i];
        b[p] -= f * b[i];
    }
    for (int64_t i = 0; i < n; ++i) {
        int64_t p = parent[i];
        if (p < 0)
            b[i] = b[i] / d[i];
        else
            b[i] = (b[i] - u[i] * b[p]) / d[i];
    }
}

/* ------------------------------------------------------------------------ */
/* construction: discretisation of each cell                                 */

static void *xcalloc(size_t n, size_t s) {
    void *p = calloc(n ? n : 1, s);
    return p;
}

static int ev_cmp(const void *a_, const void *b_) {
    const orc_event *a = a_, *b = b_;
#define CMP(x, y) \
    if ((x) < (y)) return -1; \
    if ((x) > (y)) return 1;
    CMP(a->step, b->step);
    CMP(a->kind, b->kind);
    CMP(a->syn, b->syn);
    CMP(a->src, b->src);
    CMP(a->seq, b->seq);
    return 0;
}

static int sp_cmp(const void *a_, const void *b_) {
    const orc_spike *a = a_, *b = b_;
    CMP(a->gid, b->gid);
    CMP(a->step, b->step);
    return 0;
}
#undef CMP

static void ev_push(orc *s, orc_event e) {
    if (s->nev == s->capev) {
        s->capev = s->capev ? 2 * s->capev : 1024;
        s->ev = realloc(s->ev, (size_t)s->capev * sizeof(orc_event));
    }
    s->ev[s->nev++] = e;
}

/* lateral area of a cylinder piece (um^2) */
static double piece_area(double diam, double len) { return M_PI * diam * len; }

/* axial conductance (nS) of a cylinder of diameter d and length h (um),
 * resistivity Ra (ohm cm): G = pi d^2 / (4 Ra h), with um -> cm and S -> nS */
static double axial_nS(double d, double h, double Ra) { return 2.5e4 * M_PI * d * d / (Ra * h); }

orc *orc_build(int32_t ncell, const int64_t *cell_branch_begin, const int32_t *cell_n_branch,
               const double *soma_area, const uint32_t *soma_mech, const double *soma_gna,
               const double *soma_gk, const double *soma_gl, const double *soma_gpas,
               const double *soma_epas, const double *cm, const double *Ra,
               const int32_t *br_parent, const int32_t *br_n_cv, const double *br_length,
               const double *br_diam, const uint32_t *br_mech, const double *br_gna,
               const double *br_gk, const double *br_gl, const double *br_gpas,
               const double *br_epas, int64_t nsyn, const int32_t *syn_cell,
               const int32_t *syn_branch, const int32_t *syn_cvi, const double *syn_tau,
               const double *syn_e, int64_t ncon, const uint32_t *con_src,
               const uint32_t *con_syn, const int32_t *con_delay, const double *con_w,
               int64_t next, const uint32_t *ev_syn, const int64_t *ev_step, const double *ev_w,
               int64_t nic, const int32_t *ic_cell, const int32_t *ic_branch,
               const int32_t *ic_cvi, const int64_t *ic_on, const int64_t *ic_off,
               const double *ic_amp, double dt, double theta, double v0, int32_t K) {
    orc *s = xcalloc(1, sizeof(orc));
    s->ncell = ncell;
    s->dt = dt;
    s->theta = theta;
    s->v0 = v0;
    s->K = K;

    /* counts */
    s->cv_begin = xcalloc(ncell + 1, sizeof(int64_t));
    s->reg_begin = xcalloc(ncell + 1, sizeof(int64_t));
    for (int32_t c = 0; c < ncell; ++c) {
        int64_t n = 1;
        for (int32_t b = 0; b < cell_n_branch[c]; ++b) n += br_n_cv[cell_branch_begin[c] + b];
        s->cv_begin[c + 1] = s->cv_begin[c] + n;
        s->reg_begin[c + 1] = s->reg_begin[c] + 1 + cell_n_branch[c];
    }
    int64_t ncv = s->ncv = s->cv_begin[ncell];
    int64_t nreg = s->nreg = s->reg_begin[ncell];
    s->parent = xcalloc(ncv, sizeof(int64_t));
    s->cap = xcalloc(ncv, sizeof(double));
    s->sig = xcalloc(ncv, sizeof(double));
    s->has_hh = xcalloc(ncv, 1);
    s->reg_mech = xcalloc(nreg, sizeof(uint32_t));
    s->reg_gna = xcalloc(nreg, sizeof(double));
    s->reg_gk = xcalloc(nreg, sizeof(double));
    s->reg_gl = xcalloc(nreg, sizeof(double));
    s->reg_gpas = xcalloc(nreg, sizeof(double));
    s->reg_epas = xcalloc(nreg, sizeof(double));
    s->reg_cell = xcalloc(nreg, sizeof(int64_t));

    /* membrane pieces: each CV gets at most (1 + 1 + children) pieces; count
     * generously as 2 per CV plus one per branch (its first half-segment goes
     * to the parent node). */
    int64_t nbr_tot = 0;
    for (int32_t c = 0; c < ncell; ++c) nbr_tot += cell_n_branch[c];
    int64_t cap_ct = 2 * ncv + nbr_tot + 1;
    int64_t *tmp_cv = xcalloc(cap_ct, sizeof(int64_t));
    int64_t *tmp_reg = xcalloc(cap_ct, sizeof(int64_t));
    double *tmp_area = xcalloc(cap_ct, sizeof(double));
    int64_t nct = 0;

    for (int32_t c = 0; c < ncell; ++c) {
        int64_t cv0 = s->cv_begin[c], r0 = s->reg_begin[c];
        int64_t bb = cell_branch_begin[c];
        int32_t nb = cell_n_branch[c];
        double Ram = Ra[c];
        /* region 0: soma (READING: one isopotential node of given area) */
        s->reg_mech[r0] = soma_mech[c];
        s->reg_gna[r0] = soma_gna[c];
        s->reg_gk[r0] = soma_gk[c];
        s->reg_gl[r0] = soma_gl[c];
        s->reg_gpas[r0] = soma_gpas[c];
        s->reg_epas[r0] = soma_epas[c];
        s->reg_cell[r0] = c;
        s->parent[cv0] = -1;
        s->sig[cv0] = 0.0;
        tmp_cv[nct] = cv0;
        tmp_reg[nct] = r0;
        tmp_area[nct] = soma_area[c];
        ++nct;
        /* first CV of every branch, in branch order */
        int64_t *first = xcalloc(nb + 1, sizeof(int64_t));
        int64_t next_cv = cv0 + 1;
        for (int32_t b = 0; b < nb; ++b) {
            first[b] = next_cv;
            next_cv += br_n_cv[bb + b];
        }
        for (int32_t b = 0; b < nb; ++b) {
            int64_t gb = bb + b, r = r0 + 1 + b;
            s->reg_mech[r] = br_mech[gb];
            s->reg_gna[r] = br_gna[gb];
            s->reg_gk[r] = br_gk[gb];
            s->reg_gl[r] = br_gl[gb];
            s->reg_gpas[r] = br_gpas[gb];
            s->reg_epas[r] = br_epas[gb];
            s->reg_cell[r] = c;
            int32_t n = br_n_cv[gb];
            double L = br_length[gb], dm = br_diam[gb], h = L / n;
            /* READING: nodes at x_k = k h (k = 1..n) from the proximal end;
             * x_0 is the parent node: the soma, or the parent branch's last
             * node.  CV of node k = [x_k - h/2, x_k + h/2] clipped to the
             * branch; the parent node owns [0, h/2]. */
            int32_t pb = br_parent[gb];
            int64_t pnode = (pb < 0) ? cv0 : first[pb] + br_n_cv[bb + pb] - 1;
            tmp_cv[nct] = pnode;
            tmp_reg[nct] = r;
            tmp_area[nct] = piece_area(dm, 0.5 * h);
            ++nct;
            for (int32_t k = 1; k <= n; ++k) {
                int64_t i = first[b] + (k - 1);
                s->parent[i] = (k == 1) ? pnode : i - 1;
                s->sig[i] = axial_nS(dm, h, Ram);
                /* proximal half [x_k - h/2, x_k] */
                double len = 0.5 * h;
                /* distal half [x_k, x_k + h/2], absent at the branch end */
                if (k < n) len += 0.5 * h;
                tmp_cv[nct] = i;
                tmp_reg[nct] = r;
                tmp_area[nct] = piece_area(dm, len);
                ++nct;
            }
        }
        free(first);
    }

    /* group the pieces per CV (stable in insertion order) */
    s->ct_begin = xcalloc(ncv + 1, sizeof(int64_t));
    for (int64_t k = 0; k < nct; ++k) s->ct_begin[tmp_cv[k] + 1]++;
    for (int64_t i = 0; i < ncv; ++i) s->ct_begin[i + 1] += s->ct_begin[i];
    s->ct_reg = xcalloc(nct, sizeof(int64_t));
    s->ct_area = xcalloc(nct, sizeof(double));
    int64_t *fill = xcalloc(ncv, sizeof(int64_t));
    for (int64_t k = 0; k < nct; ++k) {
        int64_t i = tmp_cv[k], at = s->ct_begin[i] + fill[i]++;
        s->ct_reg[at] = tmp_reg[k];
        s->ct_area[at] = tmp_area[k];
    }
    free(fill);
    free(tmp_cv);
    free(tmp_reg);
    free(tmp_area);

    /* capacitance and hh presence (READING: c_i = c_m x total area; a
     * mechanism acts on the area of the CV that carries it) */
    for (int32_t c = 0; c < ncell; ++c)
        for (int64_t i = s->cv_begin[c]; i < s->cv_begin[c + 1]; ++i) {
            double a = 0.0;
            for (int64_t k = s->ct_begin[i]; k < s->ct_begin[i + 1]; ++k) {
                a += s->ct_area[k];
                if (s->reg_mech[s->ct_reg[k]] & MECH_HH) s->has_hh[i] = 1;
            }
            /* uF/cm^2 * um^2 -> pF */
            s->cap[i] = 0.01 * cm[c] * a;
        }

    /* cell-local parent indices and off-diagonal entries of the matrix */
    s->lpar = xcalloc(ncv, sizeof(int64_t));
    s->uoff = xcalloc(ncv, sizeof(double));
    for (int32_t c = 0; c < ncell; ++c)
        for (int64_t i = s->cv_begin[c]; i < s->cv_begin[c + 1]; ++i) {
            s->lpar[i] = s->parent[i] < 0 ? -1 : s->parent[i] - s->cv_begin[c];
            s->uoff[i] = -s->sig[i];
        }

    /* synapses */
    s->nsyn = nsyn;
    s->syn_cv = xcalloc(nsyn, sizeof(int64_t));
    s->syn_tau = xcalloc(nsyn, sizeof(double));
    s->syn_e = xcalloc(nsyn, sizeof(double));
    for (int64_t k = 0; k < nsyn; ++k) {
        int32_t c = syn_cell[k], b = syn_branch[k];
        int64_t i = s->cv_begin[c];
        if (b >= 0) {
            int64_t at = s->cv_begin[c] + 1;
            for (int32_t q = 0; q < b; ++q) at += br_n_cv[cell_branch_begin[c] + q];
            i = at + syn_cvi[k];
        }
        s->syn_cv[k] = i;
        s->syn_tau[k] = syn_tau[k];
        s->syn_e[k] = syn_e[k];
    }

    /* connections grouped by source, then by (synapse, input index) */
    s->ncon = ncon;
    s->out_begin = xcalloc(ncell + 1, sizeof(int64_t));
    for (int64_t k = 0; k < ncon; ++k) s->out_begin[con_src[k] + 1]++;
    for (int32_t c = 0; c < ncell; ++c) s->out_begin[c + 1] += s->out_begin[c];
    s->out_syn = xcalloc(ncon, sizeof(uint32_t));
    s->out_src = xcalloc(ncon, sizeof(uint32_t));
    s->out_delay = xcalloc(ncon, sizeof(int32_t));
    s->out_w = xcalloc(ncon, sizeof(double));
    s->out_id = xcalloc(ncon, sizeof(int64_t));
    int64_t *ofill = xcalloc(ncell, sizeof(int64_t));
    for (int64_t k = 0; k < ncon; ++k) {
        uint32_t src = con_src[k];
        int64_t at = s->out_begin[src] + ofill[src]++;
        s->out_syn[at] = con_syn[k];
        s->out_src[at] = src;
        s->out_delay[at] = con_delay[k];
        s->out_w[at] = con_w[k];
        s->out_id[at] = k;
    }
    free(ofill);

    /* current clamps */
    s->nic = nic;
    s->ic_cv = xcalloc(nic, sizeof(int64_t));
    s->ic_on = xcalloc(nic, sizeof(int64_t));
    s->ic_off = xcalloc(nic, sizeof(int64_t));
    s->ic_amp = xcalloc(nic, sizeof(double));
    for (int64_t k = 0; k < nic; ++k) {
        int32_t c = ic_cell[k], b = ic_branch[k];
        int64_t i = s->cv_begin[c];
        if (b >= 0) {
            int64_t at = s->cv_begin[c] + 1;
            for (int32_t q = 0; q < b; ++q) at += br_n_cv[cell_branch_begin[c] + q];
            i = at + ic_cvi[k];
        }
        s->ic_cv[k] = i;
        s->ic_on[k] = ic_on[k];
        s->ic_off[k] = ic_off[k];
        s->ic_amp[k] = ic_amp[k];
    }

    /* external events */
    for (int64_t k = 0; k < next; ++k) {
        orc_event e = {ev_step[k], 1, ev_syn[k], 0xffffffffu, k, ev_w[k]};
        ev_push(s, e);
    }
    if (s->nev > 1) qsort(s->ev, (size_t)s->nev, sizeof(orc_event), ev_cmp);

    /* state (READING: V = v_init; gates at steady state; g = 0) */
    s->V = xcalloc(ncv, sizeof(double));
    s->m = xcalloc(ncv, sizeof(double));
    s->h = xcalloc(ncv, sizeof(double));
    s->n = xcalloc(ncv, sizeof(double));
    s->g = xcalloc(nsyn, sizeof(double));
    s->d = xcalloc(ncv, sizeof(double));
    s->rhs = xcalloc(ncv, sizeof(double));
    s->I = xcalloc(ncv, sizeof(double));
    double r[6];
    orc_hh_rates(v0, r);
    for (int64_t i = 0; i < ncv; ++i) {
        s->V[i] = v0;
        s->m[i] = r[0] / (r[0] + r[1]);
        s->h[i] = r[2] / (r[2] + r[3]);
        s->n[i] = r[4] / (r[4] + r[5]);
    }
    return s;
}

void orc_free(orc *s) {
    if (!s) return;
    void *ps[] = {s->cv_begin, s->reg_begin, s->parent, s->cap, s->sig, s->ct_begin, s->ct_reg,
                  s->ct_area, s->has_hh, s->lpar, s->uoff, s->reg_mech, s->reg_gna, s->reg_gk, s->reg_gl,
                  s->reg_gpas, s->reg_epas, s->reg_cell, s->syn_cv, s->syn_tau, s->syn_e,
                  s->out_begin, s->out_syn, s->out_src, s->out_delay, s->out_w, s->out_id,
                  s->ic_cv, s->ic_on, s->ic_off, s->ic_amp, s->V, s->m, s->h, s->n, s->g,
                  s->ev, s->sp, s->rec, s->d, s->rhs, s->I, s->tcell, s->kcell, s->out_delay_ms, s->syn_cell,
                  s->csyn_begin, s->csyn, s->tev, s->tev_begin, s->tev_end, s->tev_head,
                  s->gen_begin, s->gen_mech, s->gen_w, s->gen_p, s->gen_s};
    for (size_t k = 0; k < sizeof(ps) / sizeof(ps[0]); ++k) free(ps[k]);
    free(s);
}

/* ------------------------------------------------------------------------ */
/* one time step                                                             */

/* the further density mechanisms (defined below) */
static double gen_current(int32_t mech, const double *p, const double *st, double v);
static void gen_states(int32_t mech, const double *p, double *st, double v, double dt);

/* membrane current I_i (pA, outward positive) of every CV at the present V,
 * gates and synaptic conductances, minus injected current (eq. 2a) */
static void currents(orc *s, int64_t n_step) {
    for (int64_t i = 0; i < s->ncv; ++i) {
        double v = s->V[i], I = 0.0;
        for (int64_t k = s->ct_begin[i]; k < s->ct_begin[i + 1]; ++k) {
            int64_t r = s->ct_reg[k];
            /* S/cm^2 * um^2 -> nS */
            double a10 = 10.0 * s->ct_area[k];
            uint32_t mech = s->reg_mech[r];
            if (mech & MECH_PAS) I += a10 * s->reg_gpas[r] * (v - s->reg_epas[r]);
            if (mech & MECH_HH) {
                double m = s->m[i], h = s->h[i], n = s->n[i];
                I += a10 * s->reg_gna[r] * m * m * m * h * (v - E_NA);
                I += a10 * s->reg_gk[r] * n * n * n * n * (v - E_K);
                I += a10 * s->reg_gl[r] * (v - E_L);
            }
        }
        if (s->gen_begin)
            for (int64_t q = s->gen_begin[i]; q < s->gen_begin[i + 1]; ++q)
                I += s->gen_w[q] * gen_current(s->gen_mech[q], s->gen_p + q * 8, s->gen_s + q * 4, v);
        s->I[i] = I;
    }
    /* READING: expsyn current g (V - e) */
    for (int64_t k = 0; k < s->nsyn; ++k) {
        int64_t i = s->syn_cv[k];
        s->I[i] += s->g[k] * (s->V[i] - s->syn_e[k]);
    }
    /* READING: a positive clamp amplitude depolarises; nA -> pA */
    for (int64_t k = 0; k < s->nic; ++k)
        if (s->ic_on[k] <= n_step && n_step < s->ic_off[k]) s->I[s->ic_cv[k]] -= 1000.0 * s->ic_amp[k];
}

static void deliver_events(orc *s, int64_t n_step) {
    while (s->ev_head < s->nev && s->ev[s->ev_head].step == n_step) {
        orc_event e = s->ev[s->ev_head++];
        s->g[e.syn] += 1000.0 * e.w; /* uS -> nS */
        if (s->record_events) {
            if (s->nrec == s->caprec) {
                s->caprec = s->caprec ? 2 * s->caprec : 1024;
                s->rec = realloc(s->rec, (size_t)s->caprec * sizeof(orc_event));
            }
            s->rec[s->nrec++] = e;
        }
    }
}

static void gate_update(double *x, double a, double b, double dt) {
    double xinf = a / (a + b);
    *x = xinf + (*x - xinf) * exp(-dt * (a + b));
}

/* ------------------------------------------------------------------------ */
/* further density mechanisms, each written out from its definition (a gate
 * with first-order kinetics integrated exactly at fixed V, as the hh gates
 * are; a current density in S/cm^2 x mV):
 *   kdr:    n' = a_n (1 - n) - b_n n, a_n = 0.16 exprelr(-(V + 52)/5),
 *           b_n = 0.5 e^{-(V + 57)/40};  i = gbar n^4 (V - ek)
 *           parameters gbar 0.01, ek -90
 *   hcn:    q' = (q_inf - q)/tau_q, q_inf = 1/(1 + e^{(V - vhalf)/6}),
 *           tau_q = 50 + 200/(1 + e^{(V + 60)/10});  i = gbar q (V - eh)
 *           parameters gbar 0.0001, eh -30, vhalf -80
 *   hh_dsl: the Hodgkin-Huxley sodium, potassium and leak currents with
 *           their own densities and reversal potentials (the textbook rates
 *           of orc_hh_rates); parameters gnabar 0.12, gkbar 0.036,
 *           gl 0.0003, ena 50, ek -77, el -54.3 */

enum { ORC_GEN_KDR = 0, ORC_GEN_HCN = 1, ORC_GEN_HHDSL = 2, ORC_GEN_COUNT = 3 };

static double gen_exprelr(double x) { return (1.0 + x == 1.0) ? 1.0 : x / expm1(x); }

static const double gen_defaults[ORC_GEN_COUNT][8] = {
    {0.01, -90.0},
    {0.0001, -30.0, -80.0},
    {0.12, 0.036, 0.0003, 50.0, -77.0, -54.3},
};
static const int gen_nparams[ORC_GEN_COUNT] = {2, 3, 6};

static double gen_current(int32_t mech, const double *p, const double *st, double v) {
    switch (mech) {
    case ORC_GEN_KDR: {
        double n = st[0];
        return p[0] * n * n * n * n * (v - p[1]);
    }
    case ORC_GEN_HCN:
        return p[0] * st[0] * (v - p[1]);
    case ORC_GEN_HHDSL: {
        double m = st[0], h = st[1], n = st[2];
        return p[0] * m * m * m * h * (v - p[3]) + p[1] * n * n * n * n * (v - p[4]) + p[2] * (v - p[5]);
    }
    }
    return 0.0;
}

static void hcn_inf_tau(const double *p, double v, double *inf, double *tau) {
    *inf = 1.0 / (1.0 + exp((v - p[2]) / 6.0));
    *tau = 50.0 + 200.0 / (1.0 + exp((v + 60.0) / 10.0));
}

/* the states after a step of dt at fixed v (dt = -1: at rest at v) */
static void gen_states(int32_t mech, const double *p, double *st, double v, double dt) {
    switch (mech) {
    case ORC_GEN_KDR: {
        double a = 0.16 * gen_exprelr(-(v + 52.0) / 5.0), b = 0.5 * exp(-(v + 57.0) / 40.0);
        if (dt < 0) st[0] = a / (a + b);
        else gate_update(&st[0], a, b, dt);
        return;
    }
    case ORC_GEN_HCN: {
        double inf, tau;
        hcn_inf_tau(p, v, &inf, &tau);
        st[0] = (dt < 0) ? inf : inf + (st[0] - inf) * exp(-dt / tau);
        return;
    }
    case ORC_GEN_HHDSL: {
        double r[6];
        orc_hh_rates(v, r);
        for (int g = 0; g < 3; ++g) {
            if (dt < 0) st[g] = r[2 * g] / (r[2 * g] + r[2 * g + 1]);
            else gate_update(&st[g], r[2 * g], r[2 * g + 1], dt);
        }
        return;
    }
    }
}

/* Densities of the further mechanisms on regions (cell, branch; branch -1
 * = the soma), parameters in the mechanism's order (n_param given, the rest
 * default).  Every CV piece on such a region gets an instance with the
 * piece's area, at rest at the CV's present V.  Returns 0, or -1 for a bad
 * entry. */
int orc_set_densities(orc *s, int64_t n, const int32_t *cell, const int32_t *branch, const int32_t *mech,
                      const int32_t *n_param, const double *param) {
    for (int64_t q = 0; q < n; ++q) {
        if (cell[q] < 0 || cell[q] >= s->ncell || mech[q] < 0 || mech[q] >= ORC_GEN_COUNT) return -1;
        if (branch[q] < -1 || s->reg_begin[cell[q]] + 1 + branch[q] >= s->reg_begin[cell[q] + 1]) return -1;
        if (n_param[q] < 0 || n_param[q] > gen_nparams[mech[q]]) return -1;
    }
    s->gen_begin = xcalloc((size_t)s->ncv + 1, sizeof(int64_t));
    int64_t cnt = 0;
    for (int pass = 0; pass < 2; ++pass) {
        cnt = 0;
        for (int64_t i = 0; i < s->ncv; ++i) {
            if (pass == 1) s->gen_begin[i] = cnt;
            for (int64_t k = s->ct_begin[i]; k < s->ct_begin[i + 1]; ++k)
                for (int64_t q = 0; q < n; ++q) {
                    if (s->reg_begin[cell[q]] + 1 + branch[q] != s->ct_reg[k]) continue;
                    if (pass == 1) {
                        s->gen_mech[cnt] = mech[q];
                        s->gen_w[cnt] = 10.0 * s->ct_area[k];
                        for (int j = 0; j < 8; ++j)
                            s->gen_p[cnt * 8 + j] = (j < n_param[q]) ? param[q * 8 + j] : gen_defaults[mech[q]][j];
                        gen_states(mech[q], s->gen_p + cnt * 8, s->gen_s + cnt * 4, s->V[i], -1.0);
                    }
                    ++cnt;
                }
        }
        if (pass == 0) {
            s->ngen = cnt;
            s->gen_mech = xcalloc((size_t)cnt + 1, sizeof(int32_t));
            s->gen_w = xcalloc((size_t)cnt + 1, sizeof(double));
            s->gen_p = xcalloc((size_t)cnt * 8 + 1, sizeof(double));
            s->gen_s = xcalloc((size_t)cnt * 4 + 1, sizeof(double));
        }
    }
    s->gen_begin[s->ncv] = cnt;
    return 0;
}

/* a further mechanism's defaults; returns its parameter count */
int orc_gen_defaults(int32_t mech, double *out) {
    if (mech < 0 || mech >= ORC_GEN_COUNT) return -1;
    for (int j = 0; j < 8; ++j) out[j] = gen_defaults[mech][j];
    return gen_nparams[mech];
}

int64_t orc_gen_count(orc *s) { return s->ngen; }

/* the states of every instance, [ngen][4] (for tests) */
int orc_gen_states(orc *s, double *st) {
    for (int64_t q = 0; q < s->ngen * 4; ++q) st[q] = s->gen_s[q];
    return (int)s->ngen;
}

static void record_spike(orc *s, uint32_t gid, int64_t step, double t) {
    if (s->nsp == s->capsp) {
        s->capsp = s->capsp ? 2 * s->capsp : 1024;
        s->sp = realloc(s->sp, (size_t)s->capsp * sizeof(orc_spike));
    }
    orc_spike x = {gid, step, t};
    s->sp[s->nsp++] = x;
}

/* exchange at an epoch end: spikes of the epoch, sorted by (gid, step), are
 * walked against the source's connections; each match becomes an event at
 * spike step + delay (Sec. IV-A) */
static void exchange(orc *s) {
    int64_t b = s->sp_epoch_begin, e = s->nsp;
    if (e - b > 1) qsort(s->sp + b, (size_t)(e - b), sizeof(orc_spike), sp_cmp);
    int64_t before = s->nev;
    for (int64_t k = b; k < e; ++k) {
        uint32_t src = s->sp[k].gid;
        for (int64_t c = s->out_begin[src]; c < s->out_begin[src + 1]; ++c) {
            orc_event ev = {s->sp[k].step + s->out_delay[c], 0, s->out_syn[c], src, s->out_id[c],
                            s->out_w[c]};
            ev_push(s, ev);
        }
    }
    if (s->nev > before)
        qsort(s->ev + s->ev_head, (size_t)(s->nev - s->ev_head), sizeof(orc_event), ev_cmp);
    s->sp_epoch_begin = s->nsp;
}

/* advance every cell by one step n -> n+1 */
static void step_once(orc *s) {
    int64_t n = s->step;
    double dt = s->dt;
    deliver_events(s, n);
    currents(s, n);
    /* assemble: d_i = c_i/dt + sum_j sigma_ij, off-diagonal -sigma,
     * rhs_i = (c_i/dt) V_i - I_i */
    for (int64_t i = 0; i < s->ncv; ++i) {
        s->d[i] = s->cap[i] / dt;
        s->rhs[i] = s->cap[i] / dt * s->V[i] - s->I[i];
    }
    for (int64_t i = 0; i < s->ncv; ++i) {
        int64_t p = s->parent[i];
        if (p < 0) continue;
        s->d[i] += s->sig[i];
        s->d[p] += s->sig[i];
    }
    for (int32_t c = 0; c < s->ncell; ++c) {
        int64_t c0 = s->cv_begin[c], nc = s->cv_begin[c + 1] - c0;
        double vs_old = s->V[c0];
        /* per-cell Hines solve on local indices */
        orc_hines_solve(nc, s->lpar + c0, s->d + c0, s->uoff + c0, s->rhs + c0);
        for (int64_t k = 0; k < nc; ++k) s->V[c0 + k] = s->rhs[c0 + k];
        /* READING: upward crossing of the threshold at the soma node */
        double vs_new = s->V[c0];
        if (vs_old < s->theta && vs_new >= s->theta)
            record_spike(s, (uint32_t)c, n + 1, (n + (s->theta - vs_old) / (vs_new - vs_old)) * dt);
    }
    /* states with the updated voltage */
    for (int64_t i = 0; i < s->ncv; ++i) {
        if (!s->has_hh[i]) continue;
        double r[6];
        orc_hh_rates(s->V[i], r);
        gate_update(&s->m[i], r[0], r[1], dt);
        gate_update(&s->h[i], r[2], r[3], dt);
        gate_update(&s->n[i], r[4], r[5], dt);
    }
    if (s->gen_begin)
        for (int64_t i = 0; i < s->ncv; ++i)
            for (int64_t q = s->gen_begin[i]; q < s->gen_begin[i + 1]; ++q)
                gen_states(s->gen_mech[q], s->gen_p + q * 8, s->gen_s + q * 4, s->V[i], dt);
    for (int64_t k = 0; k < s->nsyn; ++k) s->g[k] *= exp(-dt / s->syn_tau[k]);
    s->step = n + 1;
    if (s->step % s->K == 0) exchange(s);
}

/* run n_steps; if probes are given, trace[p * n_steps + k] = V[probe[p]]
 * after step k */
int orc_run(orc *s, int64_t n_steps, const int64_t *probe, int64_t nprobe, double *trace) {
    for (int64_t k = 0; k < n_steps; ++k) {
        step_once(s);
        for (int64_t p = 0; p < nprobe; ++p) trace[p * n_steps + k] = s->V[probe[p]];
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* accessors                                                                 */

int64_t orc_ncv(orc *s) { return s->ncv; }
int64_t orc_step(orc *s) { return s->step; }
int64_t orc_nspikes(orc *s) { return s->nsp; }
void orc_spikes(orc *s, uint32_t *gid, int64_t *step, double *t) {
    for (int64_t k = 0; k < s->nsp; ++k) {
        gid[k] = s->sp[k].gid;
        step[k] = s->sp[k].step;
        t[k] = s->sp[k].t;
    }
}
void orc_get_state(orc *s, double *V, double *m, double *h, double *n, double *g) {
    memcpy(V, s->V, (size_t)s->ncv * sizeof(double));
    memcpy(m, s->m, (size_t)s->ncv * sizeof(double));
    memcpy(h, s->h, (size_t)s->ncv * sizeof(double));
    memcpy(n, s->n, (size_t)s->ncv * sizeof(double));
    memcpy(g, s->g, (size_t)s->nsyn * sizeof(double));
}
void orc_set_voltage(orc *s, const double *V) { memcpy(s->V, V, (size_t)s->ncv * sizeof(double)); }
void orc_set_gates(orc *s, const double *m, const double *h, const double *n) {
    memcpy(s->m, m, (size_t)s->ncv * sizeof(double));
    memcpy(s->h, h, (size_t)s->ncv * sizeof(double));
    memcpy(s->n, n, (size_t)s->ncv * sizeof(double));
}
/* per-CV discretisation: parent (global, -1 at soma), capacitance pF,
 * axial conductance to parent nS, total area um^2 */
void orc_cv_info(orc *s, int64_t *parent, double *cap, double *sig, double *area) {
    for (int64_t i = 0; i < s->ncv; ++i) {
        parent[i] = s->parent[i];
        cap[i] = s->cap[i];
        sig[i] = s->sig[i];
        double a = 0.0;
        for (int64_t k = s->ct_begin[i]; k < s->ct_begin[i + 1]; ++k) a += s->ct_area[k];
        area[i] = a;
    }
}
/* membrane current of every CV at the present state (pA), step index n for
 * clamps; used by the charge-conservation pin */
void orc_membrane_current(orc *s, int64_t n_step, double *I) {
    currents(s, n_step);
    memcpy(I, s->I, (size_t)s->ncv * sizeof(double));
}

/* theta[region][0..2] = (gbar_na, gbar_k, g_pas), regions in cell order,
 * soma first */
void orc_set_params(orc *s, const double *theta) {
    for (int64_t r = 0; r < s->nreg; ++r) {
        s->reg_gna[r] = theta[3 * r + 0];
        s->reg_gk[r] = theta[3 * r + 1];
        s->reg_gpas[r] = theta[3 * r + 2];
    }
}

/* ------------------------------------------------------------------------ */
/* discrete adjoint (the paper has no gradients; this differentiates exactly
 * the scheme above).  Forward: run n_steps recording every state and every
 * delivered event, with the spike exchange active; the events are then fixed
 * inputs.  Loss gradient dL/dtrace[c * n_steps + k] = dL/dV_soma(c) after
 * step k.  Output: grad[region][0..2] for (gbar_na, gbar_k, g_pas). The trace
 * of the forward run is written to trace[c * n_steps + k] if non-null.
 * Memory: the whole trajectory is kept (meant for small test models). */
int orc_adjoint(orc *s, int64_t n_steps, const double *dLdtrace, double *grad, double *trace) {
    if (s->gen_begin) return -3; /* the further mechanisms have no adjoint here */
    int64_t ncv = s->ncv, nsyn = s->nsyn, N = n_steps;
    double dt = s->dt;
    int64_t step0 = s->step;
    double *Vs = malloc((size_t)(N + 1) * ncv * sizeof(double));
    double *ms = malloc((size_t)(N + 1) * ncv * sizeof(double));
    double *hs = malloc((size_t)(N + 1) * ncv * sizeof(double));
    double *ns = malloc((size_t)(N + 1) * ncv * sizeof(double));
    double *gs = malloc((size_t)(N + 1) * (nsyn ? nsyn : 1) * sizeof(double)); /* post-event g */
    if (!Vs || !ms || !hs || !ns || !gs) return -2;
    for (int64_t k = 0; k < N; ++k) {
        memcpy(Vs + k * ncv, s->V, ncv * sizeof(double));
        memcpy(ms + k * ncv, s->m, ncv * sizeof(double));
        memcpy(hs + k * ncv, s->h, ncv * sizeof(double));
        memcpy(ns + k * ncv, s->n, ncv * sizeof(double));
        /* g after this step's events: replay delivery on a copy */
        int64_t head = s->ev_head;
        double *gk = gs + k * nsyn;
        memcpy(gk, s->g, nsyn * sizeof(double));
        while (head < s->nev && s->ev[head].step == s->step) {
            gk[s->ev[head].syn] += 1000.0 * s->ev[head].w;
            ++head;
        }
        step_once(s);
        if (trace)
            for (int32_t c = 0; c < s->ncell; ++c) trace[c * N + k] = s->V[s->cv_begin[c]];
    }
    memcpy(Vs + N * ncv, s->V, ncv * sizeof(double));
    (void)step0;

    /* reverse sweep */
    double *aV = calloc(ncv, sizeof(double));
    double *am = calloc(ncv, sizeof(double)), *ah = calloc(ncv, sizeof(double)),
           *an = calloc(ncv, sizeof(double));
    double *w = calloc(ncv, sizeof(double)), *dd = calloc(ncv, sizeof(double));
    double *gdiag = calloc(ncv, sizeof(double));
    memset(grad, 0, (size_t)s->nreg * 3 * sizeof(double));
    for (int32_t c = 0; c < s->ncell; ++c) aV[s->cv_begin[c]] = dLdtrace[c * N + (N - 1)];

    for (int64_t k = N - 1; k >= 0; --k) {
        const double *V0 = Vs + k * ncv, *V1 = Vs + (k + 1) * ncv;
        const double *m0 = ms + k * ncv, *h0 = hs + k * ncv, *n0 = ns + k * ncv;
        const double *g0 = gs + k * nsyn;
        /* adjoint of V^{k+1} through the gate update x^{k+1} = Phi(x^k, V^{k+1}) */
        for (int64_t i = 0; i < ncv; ++i) {
            w[i] = aV[i];
            if (!s->has_hh[i]) continue;
            double r[6], dr[6];
            orc_hh_rates(V1[i], r);
            orc_hh_rates_dv(V1[i], dr);
            const double x0[3] = {m0[i], h0[i], n0[i]};
            double *ax[3] = {&am[i], &ah[i], &an[i]};
            for (int q = 0; q < 3; ++q) {
                double a = r[2 * q], b = r[2 * q + 1], da = dr[2 * q], db = dr[2 * q + 1];
                double sum = a + b, E = exp(-dt * sum), xinf = a / sum;
                double dxinf = (da * b - a * db) / (sum * sum);
                double dPhi = dxinf * (1.0 - E) + (x0[q] - xinf) * E * (-dt * (da + db));
                w[i] += dPhi * *ax[q];
                *ax[q] *= E; /* d Phi / d x^k */
            }
        }
        /* w = A^{-1} (adjoint of V^{k+1});  A symmetric */
        for (int64_t i = 0; i < ncv; ++i) dd[i] = s->cap[i] / dt;
        for (int64_t i = 0; i < ncv; ++i) {
            int64_t p = s->parent[i];
            if (p < 0) continue;
            dd[i] += s->sig[i];
            dd[p] += s->sig[i];
        }
        for (int32_t c = 0; c < s->ncell; ++c) {
            int64_t c0 = s->cv_begin[c], nc = s->cv_begin[c + 1] - c0;
            orc_hines_solve(nc, s->lpar + c0, dd + c0, s->uoff + c0, w + c0);
        }
        /* dI/dV (diagonal) at step k, and the parameter and gate terms */
        for (int64_t i = 0; i < ncv; ++i) gdiag[i] = 0.0;
        for (int64_t q = 0; q < nsyn; ++q) gdiag[s->syn_cv[q]] += g0[q];
        for (int64_t i = 0; i < ncv; ++i) {
            double v = V0[i], m = m0[i], h = h0[i], n = n0[i], wi = w[i];
            double dIdV = gdiag[i], dIdm = 0.0, dIdh = 0.0, dIdn = 0.0;
            for (int64_t q = s->ct_begin[i]; q < s->ct_begin[i + 1]; ++q) {
                int64_t r = s->ct_reg[q];
                double a10 = 10.0 * s->ct_area[q];
                uint32_t mech = s->reg_mech[r];
                if (mech & MECH_PAS) {
                    dIdV += a10 * s->reg_gpas[r];
                    grad[3 * r + 2] -= a10 * (v - s->reg_epas[r]) * wi;
                }
                if (mech & MECH_HH) {
                    dIdV += a10 * (s->reg_gna[r] * m * m * m * h + s->reg_gk[r] * n * n * n * n +
                                   s->reg_gl[r]);
                    dIdm += a10 * s->reg_gna[r] * 3.0 * m * m * h * (v - E_NA);
                    dIdh += a10 * s->reg_gna[r] * m * m * m * (v - E_NA);
                    dIdn += a10 * s->reg_gk[r] * 4.0 * n * n * n * (v - E_K);
                    grad[3 * r + 0] -= a10 * m * m * m * h * (v - E_NA) * wi;
                    grad[3 * r + 1] -= a10 * n * n * n * n * (v - E_K) * wi;
                }
            }
            aV[i] = s->cap[i] / dt * wi - dIdV * wi;
            am[i] -= dIdm * wi;
            ah[i] -= dIdh * wi;
            an[i] -= dIdn * wi;
        }
        if (k >= 1)
            for (int32_t c = 0; c < s->ncell; ++c) aV[s->cv_begin[c]] += dLdtrace[c * N + (k - 1)];
    }
    free(Vs);
    free(ms);
    free(hs);
    free(ns);
    free(gs);
    free(aV);
    free(am);
    free(ah);
    free(an);
    free(w);
    free(dd);
    free(gdiag);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Variable time step (Sec. II: a spike's arrival changes a synapse's state
 * at once, so the step is shortened as needed for every such update to fall
 * at the beginning of a step).  Every cell keeps its own time.  Inputs are
 * continuous: external event times and connection delays in ms; a spike
 * carries its threshold crossing time interpolated within the step, and its
 * events arrive at that time plus the delay.
 * READING (the paper states the rule, not the procedure): the steps end on
 * the grid k dt unless an event comes first: from its time t in
 * [k dt, (k+1) dt) a cell steps to min((k+1) dt, its next event's time),
 * after applying every event due at or before t, and a full step from k dt
 * to (k+1) dt has length dt exactly.  An epoch is K steps of the grid (K dt
 * at most the minimum delay) and its spikes are exchanged at its end, so the
 * epoch length does not change the run.  The matrix C/dt' + L is assembled
 * and solved for each step's length dt'; gates and synapses decay over dt'.
 * Current clamps are not part of this mode. */

static int tev_cmp(const void *a_, const void *b_) {
    const orc_tev *a = a_, *b = b_;
#define CMP(x, y) \
    if ((x) < (y)) return -1; \
    if ((x) > (y)) return 1;
    CMP(a->cell, b->cell);
    CMP(a->t, b->t);
    CMP(a->kind, b->kind);
    CMP(a->syn, b->syn);
    CMP(a->src, b->src);
    CMP(a->seq, b->seq);
#undef CMP
    return 0;
}

static void tev_push(orc *s, orc_tev e) {
    if (s->ntev == s->captev) {
        s->captev = s->captev ? 2 * s->captev : 1024;
        s->tev = realloc(s->tev, (size_t)s->captev * sizeof(orc_tev));
    }
    s->tev[s->ntev++] = e;
}

/* Switch to the variable-step mode: connection delays (ms, input order),
 * external events (synapse, time ms, weight uS) replacing the step-indexed
 * ones, epoch length K_ep (steps).  Every cell starts at time 0.  Returns 0,
 * -1 if the model has current clamps, -2 if the epoch exceeds a delay. */
int orc_set_varstep(orc *s, const double *con_delay_ms, int64_t next, const uint32_t *ev_syn,
                    const double *ev_t, const double *ev_w, int64_t K_ep) {
    if (s->nic > 0) return -1;
    if (s->gen_begin) return -3; /* the further mechanisms run with the fixed step only */
    for (int64_t k = 0; k < s->ncon; ++k)
        if (!(con_delay_ms[k] >= (double)K_ep * s->dt)) return -2; /* an epoch is at most the minimum delay */
    s->varstep = 1;
    s->K_ep = K_ep;
    s->k_now = 0;
    s->tcell = xcalloc((size_t)s->ncell, sizeof(double));
    s->kcell = xcalloc((size_t)s->ncell, sizeof(int64_t));
    s->out_delay_ms = xcalloc((size_t)s->ncon, sizeof(double));
    for (int64_t c = 0; c < s->ncon; ++c) s->out_delay_ms[c] = con_delay_ms[s->out_id[c]];
    /* the cell of each synapse, and each cell's synapses */
    s->syn_cell = xcalloc((size_t)s->nsyn, sizeof(int32_t));
    s->csyn_begin = xcalloc((size_t)s->ncell + 1, sizeof(int64_t));
    s->csyn = xcalloc((size_t)s->nsyn, sizeof(int64_t));
    for (int64_t k = 0; k < s->nsyn; ++k) {
        int32_t c = 0;
        while (s->cv_begin[c + 1] <= s->syn_cv[k]) ++c;
        s->syn_cell[k] = c;
        s->csyn_begin[c + 1]++;
    }
    for (int32_t c = 0; c < s->ncell; ++c) s->csyn_begin[c + 1] += s->csyn_begin[c];
    int64_t *fill = xcalloc((size_t)s->ncell, sizeof(int64_t));
    for (int64_t k = 0; k < s->nsyn; ++k) {
        int32_t c = s->syn_cell[k];
        s->csyn[s->csyn_begin[c] + fill[c]++] = k;
    }
    free(fill);
    s->ntev = 0;
    for (int64_t k = 0; k < next; ++k) {
        orc_tev e = {s->syn_cell[ev_syn[k]], ev_t[k], 1, ev_syn[k], 0xffffffffu, k, ev_w[k]};
        tev_push(s, e);
    }
    s->tev_begin = xcalloc((size_t)s->ncell, sizeof(int64_t));
    s->tev_end = xcalloc((size_t)s->ncell, sizeof(int64_t));
    s->tev_head = xcalloc((size_t)s->ncell, sizeof(int64_t));
    return 0;
}

/* one step of length dt of cell c, from its time t (operator split of
 * Sec. II with the step's own dt) */
static void cell_step(orc *s, int32_t c, double t, double dt) {
    int64_t c0 = s->cv_begin[c], c1 = s->cv_begin[c + 1];
    for (int64_t i = c0; i < c1; ++i) {
        double v = s->V[i], I = 0.0;
        for (int64_t k = s->ct_begin[i]; k < s->ct_begin[i + 1]; ++k) {
            int64_t r = s->ct_reg[k];
            double a10 = 10.0 * s->ct_area[k];
            uint32_t mech = s->reg_mech[r];
            if (mech & MECH_PAS) I += a10 * s->reg_gpas[r] * (v - s->reg_epas[r]);
            if (mech & MECH_HH) {
                double m = s->m[i], h = s->h[i], n = s->n[i];
                I += a10 * s->reg_gna[r] * m * m * m * h * (v - E_NA);
                I += a10 * s->reg_gk[r] * n * n * n * n * (v - E_K);
                I += a10 * s->reg_gl[r] * (v - E_L);
            }
        }
        s->I[i] = I;
    }
    for (int64_t q = s->csyn_begin[c]; q < s->csyn_begin[c + 1]; ++q) {
        int64_t k = s->csyn[q], i = s->syn_cv[k];
        s->I[i] += s->g[k] * (s->V[i] - s->syn_e[k]);
    }
    for (int64_t i = c0; i < c1; ++i) {
        s->d[i] = s->cap[i] / dt;
        s->rhs[i] = s->cap[i] / dt * s->V[i] - s->I[i];
    }
    for (int64_t i = c0; i < c1; ++i) {
        int64_t p = s->parent[i];
        if (p < 0) continue;
        s->d[i] += s->sig[i];
        s->d[p] += s->sig[i];
    }
    double vs_old = s->V[c0];
    orc_hines_solve(c1 - c0, s->lpar + c0, s->d + c0, s->uoff + c0, s->rhs + c0);
    for (int64_t i = c0; i < c1; ++i) s->V[i] = s->rhs[i];
    double vs_new = s->V[c0];
    /* READING: the crossing time interpolated linearly within the step */
    if (vs_old < s->theta && vs_new >= s->theta)
        record_spike(s, (uint32_t)c, -1, t + dt * (s->theta - vs_old) / (vs_new - vs_old));
    for (int64_t i = c0; i < c1; ++i) {
        if (!s->has_hh[i]) continue;
        double r[6];
        orc_hh_rates(s->V[i], r);
        gate_update(&s->m[i], r[0], r[1], dt);
        gate_update(&s->h[i], r[2], r[3], dt);
        gate_update(&s->n[i], r[4], r[5], dt);
    }
    for (int64_t q = s->csyn_begin[c]; q < s->csyn_begin[c + 1]; ++q) {
        int64_t k = s->csyn[q];
        s->g[k] *= exp(-dt / s->syn_tau[k]);
    }
    s->nvsteps++;
}

/* cell c from its time to grid point k_end */
static void cell_advance(orc *s, int32_t c, int64_t k_end) {
    while (s->kcell[c] < k_end) {
        double t = s->tcell[c];
        int64_t k = s->kcell[c];
        int64_t *head = &s->tev_head[c];
        while (*head < s->tev_end[c] && s->tev[*head].t <= t) {
            orc_tev e = s->tev[(*head)++];
            s->g[e.syn] += 1000.0 * e.w; /* uS -> nS */
        }
        double grid0 = (double)k * s->dt, grid1 = (double)(k + 1) * s->dt;
        double target = grid1;
        if (*head < s->tev_end[c] && s->tev[*head].t < target) target = s->tev[*head].t;
        double h = (t == grid0 && target == grid1) ? s->dt : target - t;
        cell_step(s, c, t, h);
        s->tcell[c] = target;
        if (target == grid1) s->kcell[c] = k + 1;
    }
}

/* pending events sorted by (cell, time, kind, synapse, source, index) and
 * grouped by cell */
static void tev_group(orc *s) {
    if (s->ntev > 1) qsort(s->tev, (size_t)s->ntev, sizeof(orc_tev), tev_cmp);
    int64_t at = 0;
    for (int32_t c = 0; c < s->ncell; ++c) {
        s->tev_begin[c] = at;
        while (at < s->ntev && s->tev[at].cell == c) ++at;
        s->tev_end[c] = at;
        s->tev_head[c] = s->tev_begin[c];
    }
}

/* the delivered events out; the epoch's spikes (sorted by gid, time) walked
 * against their sources' connections into events at spike time + delay */
static void varstep_exchange(orc *s) {
    int64_t keep = 0;
    for (int32_t c = 0; c < s->ncell; ++c)
        for (int64_t k = s->tev_head[c]; k < s->tev_end[c]; ++k) s->tev[keep++] = s->tev[k];
    s->ntev = keep;
    int64_t b = s->sp_epoch_begin, e = s->nsp;
    for (int64_t k = b; k < e; ++k) {
        uint32_t src = s->sp[k].gid;
        for (int64_t q = s->out_begin[src]; q < s->out_begin[src + 1]; ++q) {
            orc_tev ev = {s->syn_cell[s->out_syn[q]], s->sp[k].t + s->out_delay_ms[q], 0, s->out_syn[q], src,
                          s->out_id[q], s->out_w[q]};
            tev_push(s, ev);
        }
    }
    s->sp_epoch_begin = s->nsp;
}

/* every cell from the common grid point to grid point k_end (time
 * k_end dt), epoch by epoch, spikes exchanged at each epoch end reached */
int orc_advance_to(orc *s, int64_t k_end) {
    if (!s->varstep) return -1;
    while (s->k_now < k_end) {
        int64_t ke = (s->k_now / s->K_ep + 1) * s->K_ep;
        int64_t stop = ke < k_end ? ke : k_end;
        tev_group(s);
        for (int32_t c = 0; c < s->ncell; ++c) cell_advance(s, c, stop);
        s->k_now = stop;
        if (stop == ke) varstep_exchange(s);
        else { /* partial epoch: drop the delivered events, keep the spikes for the epoch's end */
            int64_t keep = 0;
            for (int32_t c = 0; c < s->ncell; ++c)
                for (int64_t k = s->tev_head[c]; k < s->tev_end[c]; ++k) s->tev[keep++] = s->tev[k];
            s->ntev = keep;
        }
    }
    return 0;
}

int64_t orc_varstep_steps(orc *s) { return s->nvsteps; }
int64_t orc_varstep_grid(orc *s) { return s->k_now; }

