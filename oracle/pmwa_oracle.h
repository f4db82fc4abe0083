/*
 * pmwa_oracle.h -- serial CPU oracle for the parallelized multiple-worm
 * algorithm (PMWA, Masaki-Kato, Suzuki, Harada, Todo, Kawashima,
 * arXiv:1307.0328).
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, serial fp64
 * implementation of one PMWA Monte Carlo step for the hard-core
 * Bose-Hubbard model with the source term eta*Q, written from the paper:
 *   - vertex phase                      (pseudo code, Step 3)
 *   - worm creation / annihilation      (Eq. (worm), pseudo code Step 4)
 *   - worm scattering, N_cycle times    (Eq. (DB), Steps 5-6)
 *   - measurement                       (Step 6; Supplemental S-I)
 *   - temporal-boundary update          (Eq. (Para), Step 1)
 *   - spatial-boundary vertex update    (Eq. (ParaSpace), Step 2)
 * and, on its own, the worm law of one interval for a general local
 * operator Q = sum_alpha Q_alpha (Eq. (worm), general form, and the
 * sequence rule after it: soft-core bosons, spin S).
 * Only tests, the smoke check and the CPU-baseline leg of the benchmark
 * may load it.  It shares no code with the GPU library.
 *
 * Conventions (the discretised continuous-time representation):
 *   M = 2^ticks_log2 ticks per beta; vertices sit on integer ticks,
 *   worms on half-tick slots (slot u sits at u + 1/2).  Temporal boundary
 *   k sits just below tick T_k = floor(k*M/N_tau).  On a site, objects are
 *   ordered by (tick, vertices before the worm slot, bond id).
 *   Site id = y*Lx + x; bond id = 2*site + d (d = 0: +x, d = 1: +y).
 *
 * Canonical state (the exchange format with the GPU library):
 *   bstate[k*N + site]  uint8 occupation just above boundary k
 *   counts[k*N + site]  number of events of `site` in slab k
 *   events, slab-major then site-major then in time order:
 *     tick  int32
 *     info  uint32: bit0 = worm; bit3 = occupation just above the event;
 *                   vertex: bits1-2 = bond direction seen from this site
 *                           (0 +x, 1 +y, 2 -x, 3 -y);
 *                   worm:   bit1 = direction (1 = up, 0 = down).
 */
#ifndef PMWA_ORACLE_H
#define PMWA_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc_params {
    int32_t  Lx, Ly;             /* periodic Lx x Ly square lattice, >= 3    */
    double   beta;               /* inverse temperature                      */
    double   t, V, mu, eta;      /* hopping, n.n. repulsion, chem. pot., eta */
    int32_t  dom_x, dom_y, dom_tau; /* domain grid (extent >= 2 each)        */
    int32_t  ticks_log2;         /* M = 2^ticks_log2 ticks per beta          */
    int32_t  n_cycle;            /* <= 0: ceil(4 C / eta)                    */
    double   C;                  /* diagonal shift; NaN: default rule        */
    uint64_t seed;               /* Philox key                               */
    uint32_t chain_id;           /* Philox stream id (< 2^24)                */
    uint32_t pad_;
} orc_params;

/* Per-sweep raw measurement. */
typedef struct orc_obs {
    int64_t nv;      /* bond vertices present                       */
    int64_t nkink;   /* kinks among them                            */
    int64_t nw;      /* worms after the scattering phase            */
    int64_t occ2;    /* sum_i int n_i dtau, in half-ticks           */
    int64_t nn2;     /* sum_<ij> int n_i n_j dtau, in half-ticks    */
    double  qimp;    /* sum over intervals of l * g_sigma(eta*Delta*l) */
} orc_obs;

/* Sums over the accumulated sweeps (every sweep since create, set_state or
   orc_reset_observables), and the thermal averages per site built from them
   (the same estimators as the library's pmwa_observables):
     E       = 2 C - <nv> / (beta N)
     E_alt   = (V <nn2> - mu <occ2>) / (2 M N) - <nkink> / (beta N)
     E_eta   = E - <nw> / (beta N)
     density = <occ2> / (2 M N)
     Q       = <nw> / (beta eta N),   Q_imp = <qimp> / (M N),   b = Q_imp / 2
   err_*: standard errors of the means as if the sweeps were independent. */
typedef struct orc_summary {
    int64_t sweeps, nv, nkink, nw, occ2, nn2;
    double  qimp;
    double  nv_sq, nkink_sq, nw_sq, occ2_sq, nn2_sq, qimp_sq;
    double  E, E_alt, E_eta, density, Q, Q_imp, b;
    double  err_E, err_density, err_Q, err_Q_imp;
} orc_summary;

typedef struct orc_chain orc_chain;

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENOMEM = -2, ORC_ESTATE = -3, ORC_ECAP = -4 };

/* phases, in sweep order */
enum { ORC_PH_V = 1, ORC_PH_R = 2, ORC_PH_S = 3, ORC_PH_BT = 4,
       ORC_PH_BSX = 5, ORC_PH_BSY = 6, ORC_PH_END = 7 };

int  orc_create(const orc_params* p, orc_chain** out);
void orc_destroy(orc_chain* c);
int  orc_sweep(orc_chain* c, int64_t n_sweeps);
int  orc_phase(orc_chain* c, int phase);        /* one phase of a sweep */
int64_t orc_series(orc_chain* c, orc_obs* out, int64_t max_rows);
int  orc_flags(const orc_chain* c);              /* sticky error flags  */

/* canonical state */
int64_t orc_state_events(const orc_chain* c);
int  orc_get_state(const orc_chain* c, uint8_t* bstate, int32_t* counts,
                   int32_t* ticks, uint32_t* infos, int64_t cap,
                   uint64_t* sweep);
int  orc_set_state(orc_chain* c, const uint8_t* bstate, const int32_t* counts,
                   const int32_t* ticks, const uint32_t* infos, int64_t n_events,
                   uint64_t sweep);
int  orc_check(const orc_chain* c);            /* worldline invariants */
int  orc_observables(const orc_chain* c, orc_summary* out);
void orc_reset_observables(orc_chain* c);
/* 64-bit hash of the canonical state: with mix() the SplitMix64 finaliser
   and u = k*N + site, the sum modulo 2^64 over (k, site) of
   mix((u << 20) ^ (count << 1) ^ bstate) plus, over the site's events j,
   mix(mix((u << 15) | j) ^ (tick << 4 | info)). */
uint64_t orc_state_hash(const orc_chain* c);

/* derived quantities and tables (for pins) */
typedef struct orc_derived {
    double C, rho_max, lambda, delta;
    double wd[4];            /* diagonal weight, index sa | sc<<1         */
    double acc[4];           /* wd / rho_max                              */
    int32_t n_cycle, M, ntau;
    int32_t T[65];
} orc_derived;
int  orc_get_derived(const orc_chain* c, orc_derived* d);
int  orc_get_scatter_table(const orc_chain* c, double* tab /*16*4*4*/,
                           double* pair /*16*4*4 pair weights W[S0][i][j]*/);
double orc_vertex_weight(const orc_chain* c, int S);
double orc_fleg(const orc_chain* c, int sigma, int64_t ell);
double orc_tanh_ell(const orc_chain* c, int64_t ell);
/* Green function of b + b^+ on the current configuration for the n
   displacements (rx, ry, dt ticks) in disp (Supplemental S-I, n = 2); see the
   source */
int  orc_green(const orc_chain* c, const int32_t* disp, int n, double* out);
int  orc_poisson_table(const orc_chain* c, int k, double* cdf, int cap);
/* n-point functions on the current configuration (Supplemental S-I):
   pts holds ncorr correlators of npt points (rx, ry, dt ticks, op), op 0 =
   b + b^+, 1 = b, 2 = b^+; out[c] = (1/(N nbase)) sum over sites i and base
   times tau_j = floor(j M / nbase) of the estimator of
   < T prod_k O_k(i + r_k, tau_j + dt_k) > (a point at tick t sits at
   t + 1/4; equal times keep the listed order, first leftmost). */
int  orc_correlator(const orc_chain* c, int npt, const int32_t* pts, int ncorr, int nbase, double* out);

/* samplers driven by a Philox stream (phase, unit) of the current sweep */
int  orc_test_worms(orc_chain* c, uint32_t phase, uint32_t unit, int32_t ell,
                    int sigma, int32_t* offsets, uint8_t* dirs, int cap);
int  orc_test_choose(const double* w, int n, double u);
double orc_test_temporal_p0(const orc_chain* c, int p, int q, int64_t l1,
                            int64_t l2);

/* General local operator Q = sum_alpha Q_alpha on one site (Eq. (worm),
   general form): q[alpha][out][in] = <out|Q_alpha|in> >= 0, states 0..d-1. */
#define ORC_GQ_DMAX 8
#define ORC_GQ_AMAX 4
#define ORC_GQ_CAPMAX 255
typedef struct orc_localq {
    int32_t d, nalpha;
    double  q[ORC_GQ_AMAX][ORC_GQ_DMAX][ORC_GQ_DMAX];
} orc_localq;
/* Worms of one interval of `ell` free half-tick slots, bottom state p, top
   state q, x = lam * ell (lam = eta * beta / M): count, sorted distinct slot
   offsets in [0, ell), the type alpha and the state just above each worm,
   and a direction bit per worm, from the Philox stream with key `seed` and
   counter (word block, unit, sweep, stream << 8 | 10).  Returns n >= 0;
   ORC_ECAP when n > cap; ORC_ESTATE when q cannot be reached from p;
   ORC_EINVAL for bad arguments or x |Q| too large for 256 series terms. */
int orc_worms_general(const orc_localq* g, double lam, int64_t ell, int p, int q,
                      uint64_t seed, uint32_t stream, uint32_t sweep, uint32_t unit,
                      int cap, int32_t* slots, uint8_t* alpha, uint8_t* after, uint8_t* dirs);

/* Philox4x32-10 block */
void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
uint64_t orc_stream_word(const orc_chain* c, uint32_t phase, uint32_t unit,
                         uint64_t word_index);

#ifdef __cplusplus
}
#endif
#endif
