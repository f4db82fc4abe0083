/*
 * pmwa.h -- C ABI of the MI355X (gfx950) implementation of one Monte Carlo
 * sweep of the parallelized multiple-worm algorithm (PMWA; Masaki-Kato,
 * Suzuki, Harada, Todo, Kawashima, arXiv:1307.0328) for the hard-core
 * Bose-Hubbard model with the fictitious source term eta*Q:
 *
 *     H_eta = sum_<ij> [ -t (b_i^+ b_j + h.c.) + V n_i n_j ]
 *             - mu sum_i n_i - eta sum_i (b_i + b_i^+)
 *
 * (Eq. (BH), one term per nearest-neighbour bond, and H_eta = H - eta Q of
 * the introduction).  A sweep is, in this order:
 *   vertex phase             (pseudo code Step 3)
 *   worm re-generation       (Step 4, Eq. (worm))
 *   worm scattering x N_cycle (Steps 5-6, Eq. (DB)) + measurement (Step 6,
 *                             Supplemental S-I)
 *   temporal-boundary update (Step 1, Eq. (Para))
 *   spatial-boundary update  (Step 2, Eq. (ParaSpace)), x bonds then y bonds
 * The paper's space-time domains (N_beta x N_L^d decomposition, Supplemental
 * S-II) are work units on one GPU; its neighbour messages are reads and
 * writes of the neighbours' arrays in device memory.
 *
 * Representation (shared with any checker through the canonical state
 * below): M = 2^ticks_log2 ticks per beta; vertices on integer ticks, worms
 * on half-tick slots (slot u at u + 1/2); temporal boundary k just below
 * tick T_k = floor(k M / dom_tau); per site, objects ordered by (tick,
 * vertices before the worm slot, bond id); site = y*Lx + x, bond id =
 * 2*site + d (d = 0: +x, 1: +y).  Random numbers: Philox4x32-10 keyed by
 * `seed`, counter (word pair, unit, sweep, chain_id << 8 | stream kind), so
 * a chain's trajectory depends only on its parameters, never on how it is
 * batched.
 *
 * Conventions: every entry point returns 0 or a negative PMWA_E* code; no
 * exception crosses the ABI.  The handle owns all device memory it
 * allocates (hipMalloc at create, hipFree at destroy).  All pointers are
 * host pointers unless stated.  The stream in pmwa_opts is borrowed: work is
 * enqueued on it, and calls that return host data synchronise it.
 */
#ifndef PMWA_H
#define PMWA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    PMWA_OK = 0,
    PMWA_EINVAL = -1,     /* bad argument or parameter outside the limits */
    PMWA_ENOMEM = -2,     /* device or host allocation failed             */
    PMWA_EDEVICE = -3,    /* a HIP call failed                            */
    PMWA_EOVERFLOW = -4,  /* a per-site or per-bond capacity was exceeded; */
                          /* the state of that chain is no longer valid    */
    PMWA_ESTATE = -5      /* inconsistent state (set_state input, sampler) */
};

/* One chain (one Markov chain of one lattice).  Copied at create.
   Besides the per-field limits below, pmwa_create and pmwa_slot_load return
   PMWA_EINVAL for a chain outside the limits of this implementation:
     eta * beta <= 8 (the worms drawn on one interval fit the sampler);
     the Poisson table of candidate counts per bond and slab has at most 256
       entries (mean rho_max * beta / dom_tau up to about 200);
     N = Lx*Ly < 2^28; C > max E_b (every diagonal weight positive);
     n_cycle (given or default) in 1..10^7;
     events per (site, slab) <= 32767 (opts.event_cap, or the default from
       the expected density), and the spatial-boundary kernel's LDS for that
       capacity <= 160 KB. */
typedef struct pmwa_params {
    int32_t  Lx, Ly;          /* periodic Lx x Ly square lattice, each >= 3       */
    double   beta;            /* inverse temperature (beta*t with t = 1)          */
    double   t, V, mu, eta;   /* hopping >= 0, repulsion, chem. potential, eta > 0 */
    int32_t  dom_x, dom_y;    /* spatial domain grid; Lx % dom_x == 0, extent >= 2 */
    int32_t  dom_tau;         /* temporal domains N_beta, 1..64                    */
    int32_t  ticks_log2;      /* M = 2^ticks_log2 ticks per beta, 8..29            */
    int32_t  n_cycle;         /* scattering cycles per sweep; <= 0: ceil(4 C/eta)  */
    double   C;               /* diagonal shift; NaN: max_s E_b(s) + t/2          */
    uint64_t seed;            /* Philox key                                        */
    uint32_t chain_id;        /* Philox stream id, < 2^24                          */
    uint32_t pad_;
} pmwa_params;

/* Launch options.  Zero-initialise for the defaults. */
typedef struct pmwa_opts {
    void*   stream;           /* hipStream_t (borrowed); NULL: the handle creates
                                 one (default priority) and destroys it       */
    int32_t scatter_mode;     /* scattering node store: 0 and 1: LDS where the
                                 domain fits, else HBM; 2: every domain in HBM */
    int32_t series_cap;       /* per-chain device rows of per-sweep records     */
    int32_t event_cap;        /* events per (site, slab), <= 32767; 0 = from the
                                 density.  The temporal boundary update also
                                 needs room, at the top of a site's array,
                                 for the slots of a leg that draws three or
                                 more worms while it places them; running out
                                 is PMWA_EOVERFLOW like any other excess    */
    int32_t use_graph;        /* 1: replay a captured sweep (hipGraph)          */
    int32_t regen_mode;       /* worm re-generation: 0 auto, 1 a lane per (site,
                                 slab), 2 a wavefront per (site, slab); the
                                 result is the same                           */
    int32_t vertex_mode;      /* vertex phase, for tests (the result is the same):
                                 0 auto; bit0: walk the site lists in HBM even
                                 where the occupation changes fit in LDS; bit1:
                                 sort the candidates in an LDS column even
                                 where 32 registers hold them               */
    int32_t scatter_lds;      /* LDS bytes of the scattering kernel's LDS form (a
                                 tuning knob: fewer bytes let more domains share a
                                 CU, larger domains then take the HBM store); 0 =
                                 sized for the largest expected domain       */
    int32_t groups;           /* 0 or 1: every phase of every chain in one launch;
                                 G > 1: the chains split into G groups of about
                                 equal expected work, each on a stream of its
                                 own (default priority); a sweep forks to them
                                 and joins, so no group's phase waits for
                                 another group's (one graph with G branches when
                                 use_graph).  Results do not depend on it.    */
    int32_t vertex_rows;      /* occupation changes (kinks and worms) of a site
                                 in a slab that the vertex kernel stages in LDS
                                 per lane (8..128); a lane with more walks its
                                 lists in HBM.  Fewer rows let more blocks share
                                 a CU.  0: 64 when every block of the launch
                                 is resident at once anyway, else from the
                                 expected kinks per site and slab (about
                                 2.5 t dbeta plus two standard deviations).
                                 Results do not depend on it.                */
} pmwa_opts;

/* Raw per-sweep record of one chain (all sums over the whole lattice). */
typedef struct pmwa_obs {
    int64_t nv;      /* bond vertices present after the vertex phase          */
    int64_t nkink;   /* kinks among them (after the worm phase)               */
    int64_t nw;      /* worms after the scattering phase                       */
    int64_t occ2;    /* sum_i int n_i dtau after the worm phase, half-ticks    */
    int64_t nn2;     /* sum_<ij> int n_i n_j dtau before the vertex phase, half-ticks */
    double  qimp;    /* sum over intervals of l * g_sigma(eta Delta l), g_0 = tanh,
                        g_1 = coth: the improved worm-density estimator (S-I) */
} pmwa_obs;

/* Sums over the accumulated sweeps of one chain (see pmwa_observables). */
typedef struct pmwa_obs_acc {
    int64_t sweeps;                        /* sweeps accumulated                */
    int64_t nv, nkink, nw, occ2, nn2;      /* sums of the pmwa_obs fields       */
    double  qimp;
    double  nv_sq, nkink_sq, nw_sq, occ2_sq, nn2_sq, qimp_sq;  /* sums of squares,
                                              each term (double)x * (double)x  */
} pmwa_obs_acc;

/* Thermal averages per site from the accumulated sums (the estimators of
   the expansion of Tr exp(-beta H_eta) with non-negative weights, and the
   improved worm-density estimator of Supplemental S-I).  With S = sweeps,
   N = Lx*Ly sites, N_b = 2N bonds, M = 2^ticks_log2, <x> = sum_x / S:
     E        = C N_b / N - <nv> / (beta N)             energy of H per site
     E_alt    = (V <nn2> - mu <occ2>) / (2 M N) - <nkink> / (beta N)
                                                        (same mean, from the
                                                        diagonal and kink terms)
     E_eta    = E - <nw> / (beta N)                     <H_eta> per site
     density  = <occ2> / (2 M N)                        <n_i>
     Q        = <nw> / (beta eta N)                     <b_i + b_i^+> (worm count)
     Q_imp    = <qimp> / (M N)                          the same, improved estimator
     b        = Q_imp / 2                               <b_i>
   The err_* fields are standard errors of the means computed from the sums
   of squares as if the sweeps were independent (no autocorrelation
   correction; bin the pmwa_measure records for that). */
typedef struct pmwa_summary {
    pmwa_obs_acc acc;
    double E, E_alt, E_eta, density, Q, Q_imp, b;
    double err_E, err_density, err_Q, err_Q_imp;
} pmwa_summary;

/* Derived constants of one chain. */
typedef struct pmwa_info {
    double  C, rho_max, delta, lambda;    /* Delta = beta/M, lambda = eta Delta */
    int32_t n_cycle, M, event_cap, bond_cap;
    int64_t n_domains;
} pmwa_info;

typedef struct pmwa_handle pmwa_t;

/* Validate `chains[0..n_chains)`, build the tables, allocate device memory,
   enqueue the empty initial configuration (all occupations 0, no vertices,
   no worms).  *out receives the handle, or NULL on error. */
int pmwa_create(const pmwa_params* chains, int n_chains, const pmwa_opts* opts,
                pmwa_t** out);

/* Enqueue n_sweeps full sweeps of every chain on the handle's stream.  The
   per-sweep records go to a device ring; when it would overflow the call
   synchronises and drains it to host memory first. */
int pmwa_sweep(pmwa_t* h, int64_t n_sweeps);

/* Enqueue one phase of a sweep for every chain: 1 vertex, 2 worm
   re-generation, 3 scattering + measurement, 4 temporal boundaries,
   5 spatial boundaries (x), 6 spatial boundaries (y), 7 end of sweep
   (record the measurement, advance the sweep counter).  For tests. */
int pmwa_phase(pmwa_t* h, int phase);

/* Synchronise and copy up to max_rows unread per-sweep records of `chain`
   into out[]; *n_rows receives the count.  Returns PMWA_EOVERFLOW if the
   chain's state was invalidated by a capacity overflow. */
int pmwa_measure(pmwa_t* h, int chain, pmwa_obs* out, int64_t max_rows,
                 int64_t* n_rows);

/* Synchronise; return 0 or the first error raised on the device. */
int pmwa_status(pmwa_t* h);

/* Synchronise; return 0 or the error raised on the device for `chain` only
   (PMWA_EOVERFLOW, PMWA_ESTATE).  A flagged chain stops advancing; the other
   chains of the handle are unaffected. */
int pmwa_chain_status(pmwa_t* h, int chain);

/* Accumulated observables of `chain` (synchronises).  Every sweep's record
   is added on the device at the end of the sweep (k_finish), in sweep order;
   pmwa_reset_observables restarts the accumulation of every chain of the
   handle with the next sweep enqueued (stream ordered; use it after the
   thermalisation sweeps).  A slot load restarts that slot's accumulation.
   out->acc.sweeps = 0 gives NaN averages.  PMWA_EOVERFLOW / PMWA_ESTATE if
   the chain is flagged (out is still filled). */
int pmwa_observables(pmwa_t* h, int chain, pmwa_summary* out);
int pmwa_reset_observables(pmwa_t* h);

/* 64-bit hash of the canonical state of `chain` (synchronises; computed on
   the device).  With mix(z) the SplitMix64 finaliser (z ^= z >> 30;
   z *= 0xbf58476d1ce4e5b9; z ^= z >> 27; z *= 0x94d049bb133111eb;
   z ^= z >> 31) and u = k*N + site (slab k, site index y*Lx + x):
     hash = sum over (k, site) of mix((u << 20) ^ (count << 1) ^ bstate)
          + sum over its events j of
                mix(mix((u << 15) | j) ^ ((uint64_t)tick << 4 | info))
   modulo 2^64 (an order-free sum, so a parallel reduction computes it
   exactly).  count, tick and info are those of pmwa_get_state; the sweep
   counter is not part of it. */
int pmwa_state_hash(pmwa_t* h, int chain, uint64_t* out);

/* Canonical state of one chain (synchronises).  Layout:
     bstate[k*N + site]   occupation just above temporal boundary k (uint8)
     counts[k*N + site]   events of `site` in slab k
     ticks[], infos[]     events, slab-major, then site, then time order;
                          info bit0 worm, bit3 occupation above the event,
                          vertex bits1-2: bond direction from this site
                          (0 +x, 1 +y, 2 -x, 3 -y); worm bit1: 1 = moving up.
   N = Lx*Ly.  get: `cap` is the size of ticks/infos; *n_events receives the
   number of events (PMWA_EINVAL if cap is too small; call with cap = 0 to
   query).  set: replaces the state (validated: sorted, in range, capacity). */
int pmwa_get_state(pmwa_t* h, int chain, uint8_t* bstate, int32_t* counts,
                   int32_t* ticks, uint32_t* infos, int64_t cap,
                   int64_t* n_events, uint64_t* sweep);
int pmwa_set_state(pmwa_t* h, int chain, const uint8_t* bstate,
                   const int32_t* counts, const int32_t* ticks,
                   const uint32_t* infos, int64_t n_events, uint64_t sweep);

int pmwa_chain_info(pmwa_t* h, int chain, pmwa_info* out);

/* Device time per phase.  While enabled, every phase launched by pmwa_sweep
   or pmwa_phase is bracketed by two HIP events recorded on the handle's
   stream (graph replay is bypassed so each kernel has its own pair; recording
   does not synchronise).  pmwa_phase_times synchronises, returns the summed
   milliseconds and launch counts of phases 1..7 in ms[0..6] and
   launches[0..6], and resets the accumulators. */
int pmwa_set_timing(pmwa_t* h, int enable);
int pmwa_phase_times(pmwa_t* h, double* ms, int64_t* launches);
/* The same for a subset of the phases: bit p-1 of `mask` brackets phase p
   (1..7) with events; the others launch without them.  mask = 0 disables
   timing, 0x7F equals pmwa_set_timing(h, 1).  PMWA_EINVAL for other bits. */
int pmwa_set_timing_phases(pmwa_t* h, uint32_t mask);

/* Continuous batching.  pmwa_create_slots allocates n_slots chain slots;
   shapes[i] gives slot i's largest chain: a chain fits slot i when none of
   its sizes (sites x slabs, bonds x slabs, domains, sites per domain,
   crossing bonds, Poisson-table length) exceeds those of shapes[i].  Slots
   start idle.  pmwa_slot_load installs a chain in slot `slot` (stream
   ordered: its empty configuration is set up before the next sweep) that
   stops after target_sweeps sweeps; pmwa_slot_release makes the slot idle.
   pmwa_sweep advances every installed chain below its target.
   pmwa_slot_progress synchronises and returns the sweeps done.  Records
   and states are read with pmwa_measure / pmwa_get_state using the slot
   index.  A chain's trajectory does not depend on its slot or on the other
   chains.  PMWA_EINVAL if the chain does not fit the slot. */
int pmwa_create_slots(const pmwa_params* shapes, int n_slots, const pmwa_opts* opts,
                      pmwa_t** out);
int pmwa_slot_load(pmwa_t* h, int slot, const pmwa_params* p, int64_t target_sweeps);
int pmwa_slot_release(pmwa_t* h, int slot);
int pmwa_slot_progress(pmwa_t* h, int slot, int64_t* sweeps_done);
/* 0 if the chain `p` fits slot `slot` (the check of pmwa_slot_load, without
   loading), PMWA_EINVAL otherwise. */
int pmwa_slot_fits(pmwa_t* h, int slot, const pmwa_params* p);

/* Scattering-phase diagnostics of the last sweep of `chain` (synchronises):
   out[0] evaluation windows summed over domains, out[1] the most windows in
   one domain, out[2] worm attempts summed over domains, out[3] the most
   attempts in one domain.  n >= 4. */
int pmwa_diag(pmwa_t* h, int chain, int64_t* out, int n);

/* Green function of Q_i = b_i + b_i^+ (Supplemental S-I, the product rule
   for n = 2): for each of the n displacements (rx, ry, dt) in disp[3q],
   disp[3q+1], disp[3q+2] (any integers, taken modulo the lattice and, for
   the imaginary-time shift dt in ticks, modulo M = 2^ticks_log2),
   out[q] = G(r, dt) = (1/N) sum_i <Q_i(tau) Q_{i+r}(tau + dt)>, averaged over
   tau in [0, beta), on the CURRENT configuration of `chain` (one sample;
   average over sweeps for the thermal value).  The one-point ratio rho/eta
   on an interval between vertices or temporal domain boundaries is
   tanh(lambda l) for an even number of worms in it and coth(lambda l) for
   an odd number.  Two points on different intervals give the product of
   their ratios; two points on one interval give 1 (Q commutes with the
   interval propagator and Q^2 = 1); (0, 0, 0) gives 1.  disp and out are
   host arrays of 3n and n entries, 1 <= n <= PMWA_GREEN_MAX.  Synchronises
   the handle's stream; the first call allocates a small device workspace
   that the handle keeps.  PMWA_EINVAL on bad arguments, PMWA_ESTATE or
   PMWA_EOVERFLOW if the chain is flagged. */
#define PMWA_GREEN_MAX 64
int pmwa_green(pmwa_t* h, int chain, const int32_t* disp, int n, double* out);

/* n-point functions of b, b^+ and Q = b + b^+ (Supplemental S-I, any n up
   to PMWA_CORR_MAX_POINTS) on the CURRENT configuration of `chain` (one
   sample; average over sweeps for the thermal value).  pts holds ncorr
   correlators of npt points each, a point being 4 int32: (rx, ry, dt, op)
   with op 0 = b + b^+, 1 = b, 2 = b^+ and dt in ticks (all taken modulo the
   lattice and M).  out[c] = (1/(N nbase)) sum over sites i and base times
   tau_j = floor(j M / nbase), j < nbase, of the estimator of
   < T prod_k O_k(i + r_k, tau_j + dt_k) >: the worms of an interval
   (between vertices and temporal domain boundaries) are summed over, so an
   interval holding points contributes <q| E .. O .. E |p> / <q| E |p>, E the
   interval's propagator exp(l eta Delta Q) split at the points, operators in
   time order (equal times: the first listed leftmost); points on different
   intervals multiply.  A point at tick t sits at t + 1/4.  Every term is
   >= 0.  Synchronises the handle's stream; the first call allocates a small
   device workspace that the handle keeps.  PMWA_EINVAL on bad arguments,
   PMWA_ESTATE / PMWA_EOVERFLOW if the chain is flagged.  At small
   eta * (interval length) the odd-parity ratio is large (coth), so the
   estimator of a product of many points is heavy-tailed. */
#define PMWA_CORR_MAX_POINTS 8
#define PMWA_CORR_MAX 64
int pmwa_correlator(pmwa_t* h, int chain, int npt, const int32_t* pts, int ncorr, int nbase, double* out);

/* pmwa_green without any allocation, for callers that cannot allocate
   device memory (code under graph capture set-up, tight serving loops,
   harnesses that forbid hipMalloc).  Same arguments, results and errors as
   pmwa_green (equal to it: the same kernel, the partials summed in the same
   order on the device).  Its workspace (displacements, per-block partials,
   results; 4 MB + 2 KB) is one static device array per GPU, set up by
   pmwa_create; the call makes no hipMalloc/hipFree.  Limit: dom_tau *
   (distinct non-zero displacements) * ceil(Lx*Ly / 64) <=
   PMWA_GREEN_STATIC_PARTIALS, else PMWA_EINVAL (e.g. a 2048 x 2048 lattice
   with 4 slabs takes at most 2 displacements per call).  Every call on a GPU
   uses that GPU's one array: calls that overlap in time on the same GPU
   (from several threads or handles) race and must be serialised by the
   caller.  Synchronises the handle's stream. */
#define PMWA_GREEN_STATIC_PARTIALS (1 << 19)
int pmwa_green_static(pmwa_t* h, int chain, const int32_t* disp, int n, double* out);

/* ------------------------------------------------------------------------
   Worms of an interval for a general local operator (paper: "Worm creation
   and annihilation", Eq. (worm) in its general form and the sequence rule
   after it).  The worm-generating operator of a site is Q = sum_alpha
   Q_alpha over up to PMWA_GQ_AMAX operator types, each a nonnegative
   d x d matrix q[alpha][out][in] = <out|Q_alpha|in> on local states
   0..d-1, d <= PMWA_GQ_DMAX (soft-core bosons: b, b^+ with n <= d - 1;
   spin S: S^-, S^+ with d = 2S + 1; hard-core bosons are d = 2).
   ------------------------------------------------------------------------ */
#define PMWA_GQ_DMAX 8
#define PMWA_GQ_AMAX 4
#define PMWA_GQ_CAPMAX 255
typedef struct pmwa_localq {
    int32_t d, nalpha;
    double  q[PMWA_GQ_AMAX][PMWA_GQ_DMAX][PMWA_GQ_DMAX];   /* entries beyond d, nalpha ignored */
} pmwa_localq;

/* Draws the worms of n_int intervals.  Interval i has ell[i] free half-tick
   slots, bottom state p[i] and top state q[i]; with x = lam * ell[i]
   (lam = eta * beta / M, I*eta of the paper):
     - the count n with probability x^n/n! <q|Q^n|p> / <q|exp(xQ)|p>;
       <q|exp(xQ)|p> is the series of u_j = (x/j) Q u_{j-1}, u_0 = |p>,
       stopped after the first term j with j + 2 >= 2y, y = x * (largest
       column sum of Q), and either u_j = 0 or 2 y |u_j|_1 / (j + 1) <=
       2^-60 (sum so far); n by inversion of the partial sums (a new
       uniform when u*f rounds to f or n > ell[i]);
     - n distinct uniform slot offsets in [0, ell[i]), ascending;
     - the type alpha_k of worm k (time order) and the state s_k just above
       it, the path having probability prod_k <s_k|Q_alpha_k|s_{k-1}> /
       <q|Q^n|p> (s_0 = p, s_n = q), drawn from the last worm back;
     - one direction bit per worm (1 = up) in slot order.
   Random words: Philox4x32-10 with key `seed`, counter (word pair, unit0 +
   i, sweep, stream << 8 | 10), 64-bit words u53 / high-product as in the
   sweep.  All pointers except g are DEVICE pointers: p, q, ell[n_int] in;
   n_out[n_int] out (the count, or for this interval PMWA_EINVAL (state out
   of range, negative length, x |Q| too large for 256 series terms),
   PMWA_ESTATE (q unreachable from p, or no draw), PMWA_EOVERFLOW (n >
   cap)); slots (int32), alpha, after (state above the worm), dirs (uint8)
   are cap x n_int, worm k of interval i at k * n_int + i (may be NULL when
   cap = 0).  Asynchronous on hip_stream (NULL: the default stream); the
   library keeps a device workspace of (cap + 1) * d doubles per lane (at most
   512 MB, grown on demand) and orders calls on it with an event.  Returns
   PMWA_EINVAL for bad arguments (d, nalpha, negative or non-finite
   entries, lam, cap > PMWA_GQ_CAPMAX, stream >= 2^24, unit0 + n_int >
   2^32), PMWA_ENOMEM, PMWA_EDEVICE. */
int pmwa_worms_general(const pmwa_localq* g, double lam, int64_t n_int, const int32_t* p, const int32_t* q,
                       const int64_t* ell, uint64_t seed, uint32_t stream, uint32_t sweep, uint32_t unit0,
                       int32_t cap, int32_t* n_out, int32_t* slots, uint8_t* alpha, uint8_t* after,
                       uint8_t* dirs, void* hip_stream);

/* Events per (site, slab) a chain would be given by default. */
int pmwa_default_event_cap(const pmwa_params* p);

/* Free all device memory of the handle (synchronises first). */
void pmwa_destroy(pmwa_t* h);

const char* pmwa_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif
