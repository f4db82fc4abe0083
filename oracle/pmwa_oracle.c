/*
 * pmwa_oracle.c -- serial CPU oracle for one PMWA Monte Carlo step.
 *
 * TEST INFRASTRUCTURE ONLY (see pmwa_oracle.h).  Plain serial C, fp64,
 * compiled with -O2 -ffp-contract=off.  Every phase follows the paper's
 * pseudo code (Steps 1-6) in its own order and notation:
 *
 *   Step 3  vertex phase          orc_phase_V   (+ bond occupation integral)
 *   Step 4  worm re-generation    orc_phase_R
 *   Step 5-6 worm scattering      orc_phase_S   (+ measurement, Step 6, S-I)
 *   Step 1  temporal boundaries   orc_phase_BT  (Eq. (Para))
 *   Step 2  spatial boundaries    orc_phase_BS  (Eq. (ParaSpace))
 *
 * A sweep runs Steps 3,4,5,6 then 1,2 (a cyclic rotation of the paper's
 * order), so the measurement of Step 6 closes the worm phase.
 *
 * Representation: each site holds one dynamic array of events over the
 * whole imaginary-time circle [0, M), sorted by (tick, class, bond id),
 * class 0 = vertex, 1 = worm.  A vertex on bond (a, c = a + e_d) appears
 * in both site arrays; its four root states are the occupations just
 * below and just above it on a and c.
 */
#include "pmwa_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11)                   */
/* ------------------------------------------------------------------ */
void orc_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; r++) {
        if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        uint32_t y1 = (uint32_t)p1;
        uint32_t y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        uint32_t y3 = (uint32_t)p0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* ------------------------------------------------------------------ */
/* data                                                                */
/* ------------------------------------------------------------------ */
typedef struct {
    int32_t tick;
    uint8_t worm;     /* 1 worm, 0 vertex end                               */
    uint8_t dir;      /* vertex: 0 +x, 1 +y, 2 -x, 3 -y; worm: 1 up, 0 down */
    uint8_t up;       /* occupation just above this event                  */
} ev_t;

typedef struct { ev_t* e; int n, cap; } elist;

typedef struct { int32_t tick; uint8_t sa, sc; } newv_t;   /* new diag vertex */
typedef struct { newv_t* v; int n, cap; } vlist;

typedef struct { int32_t site, slot; } wref;   /* a worm in the S-phase list */

enum { FLAG_REDRAW = 1, FLAG_SIGMA = 2, FLAG_STATE = 4, FLAG_NOMEM = 8 };

struct orc_chain {
    orc_params p;
    int Lx, Ly, N, ntau, ex, ey, M;
    int32_t T[65];
    double delta, lambda, C, rho_max, wd[4], acc[4];
    double F[4][256];          /* expm1(lambda * v * 2^(8g)), digit v of ell */
    double* cdf;               /* [ntau][KMAX] Poisson CDF of candidate counts */
    int*    cdf_len;
    double scat[16][4][4];     /* cumulative exit table, row S0, entry leg i */
    double pairw[16][4][4];    /* directed-loop pair weights w_ij            */
    int ncycle;

    elist* site;               /* N */
    uint8_t* bstate;           /* [k*N + site] */
    vlist* bondv;              /* 2N: new diagonal vertices of this sweep    */
    uint64_t sweep;
    int flags;

    orc_obs cur;               /* measurement of the sweep in progress */
    orc_obs* series; int64_t nseries, capseries;
    orc_summary sums;          /* sums and squares of the recorded sweeps */
};

#define KMAX 1024

/* Philox counter word 3 carries (chain_id << 8) | stream kind */
enum { RNG_V = 1, RNG_R = 2, RNG_S = 3, RNG_BT = 4, RNG_BS = 5, RNG_BSL = 6 /* .. 9: the four legs */ };

/* ------------------------------------------------------------------ */
/* random stream of one unit                                           */
/* ------------------------------------------------------------------ */
typedef struct {
    uint32_t key[2], ctr[4];
    uint64_t w;        /* next word index          */
    uint64_t blk;      /* index of the cached block */
    uint32_t out[4];
    int have;
} rstream;

static void rs_init(rstream* s, const orc_chain* c, uint32_t phase, uint32_t unit)
{
    s->key[0] = (uint32_t)c->p.seed;
    s->key[1] = (uint32_t)(c->p.seed >> 32);
    s->ctr[0] = 0;
    s->ctr[1] = unit;
    s->ctr[2] = (uint32_t)c->sweep;
    s->ctr[3] = (c->p.chain_id << 8) | phase;
    s->w = 0; s->have = 0; s->blk = 0;
}

static uint64_t rs_next(rstream* s)
{
    uint64_t j = s->w >> 1;
    if (!s->have || s->blk != j) {
        uint32_t ctr[4] = { (uint32_t)j, s->ctr[1], s->ctr[2], s->ctr[3] };
        orc_philox(ctr, s->key, s->out);
        s->blk = j; s->have = 1;
    }
    uint64_t r = (s->w & 1)
        ? (((uint64_t)s->out[3] << 32) | s->out[2])
        : (((uint64_t)s->out[1] << 32) | s->out[0]);
    s->w++;
    return r;
}

/* uniform double in [0,1) with 53 random bits */
static double u53(uint64_t w) { return (double)(w >> 11) * 0x1.0p-53; }
/* uniform integer in [0, n): high word of the 128-bit product */
static uint64_t below(uint64_t w, uint64_t n)
{
    return (uint64_t)(((unsigned __int128)w * (unsigned __int128)n) >> 64);
}

uint64_t orc_stream_word(const orc_chain* c, uint32_t phase, uint32_t unit,
                         uint64_t word_index)
{
    rstream s; rs_init(&s, c, phase, unit);
    s.w = word_index;
    return rs_next(&s);
}

/* ------------------------------------------------------------------ */
/* lattice helpers                                                     */
/* ------------------------------------------------------------------ */
static int nb(const orc_chain* c, int site, int d)   /* d: 0 +x 1 +y 2 -x 3 -y */
{
    int x = site % c->Lx, y = site / c->Lx;
    switch (d) {
    case 0: x = (x + 1) % c->Lx; break;
    case 1: y = (y + 1) % c->Ly; break;
    case 2: x = (x + c->Lx - 1) % c->Lx; break;
    default: y = (y + c->Ly - 1) % c->Ly; break;
    }
    return y * c->Lx + x;
}
/* global bond id of the bond seen from `site` in relative direction d */
static int64_t bond_id(const orc_chain* c, int site, int d)
{
    if (d < 2) return 2 * (int64_t)site + d;
    return 2 * (int64_t)nb(c, site, d) + (d - 2);
}
static int dom_sp(const orc_chain* c, int site)
{
    int x = site % c->Lx, y = site / c->Lx;
    return (y / c->ey) * c->p.dom_x + (x / c->ex);
}
/* is bond (a, a + e_d), d in {0,1}, crossing a spatial domain boundary? */
static int is_cross(const orc_chain* c, int a, int d)
{
    return dom_sp(c, a) != dom_sp(c, nb(c, a, d));
}
static int slab_of(const orc_chain* c, int32_t tick)
{
    int k = 0;
    while (k + 1 < c->ntau && tick >= c->T[k + 1]) k++;
    return k;
}

/* ------------------------------------------------------------------ */
/* element functions of the worm law, from the expm1 bit table          */
/* ------------------------------------------------------------------ */
/* m = exp(lambda*ell) - 1, accumulated over the base-256 digits of ell in
   ascending order: (1+m)(1+t) - 1 = (m + t) + m t. */
static double em1(const orc_chain* c, int64_t ell)
{
    double m = 0.0;
    for (int g = 0; g < 4; g++) {
        int v = (int)((ell >> (8 * g)) & 255);
        if (v) {
            double t = c->F[g][v];
            m = (m + t) + m * t;
        }
    }
    return m;
}
/* f_0 = cosh(eta*Delta*ell), f_1 = sinh(eta*Delta*ell) (hard-core form of
   f_qp(I) = <q| exp(I eta Q) |p>, "Worm creation and annihilation") */
static double fleg(const orc_chain* c, int sigma, int64_t ell)
{
    double m = em1(c, ell);
    double d = 2.0 * (1.0 + m);
    if (sigma) return (m * (2.0 + m)) / d;
    return 1.0 + (m * m) / d;
}
static double tanh_ell(const orc_chain* c, int64_t ell)
{
    double m = em1(c, ell);
    double d = 2.0 * (1.0 + m);
    return (m * (2.0 + m)) / (d + m * m);
}
double orc_fleg(const orc_chain* c, int sigma, int64_t ell) { return fleg(c, sigma, ell); }
double orc_tanh_ell(const orc_chain* c, int64_t ell) { return tanh_ell(c, ell); }

/* vertex weights: diagonal C - E_b(s), kink t, otherwise 0.
   Root pattern S: bit0 a-below, bit1 c-below, bit2 a-above, bit3 c-above */
static double vweight(const orc_chain* c, int S)
{
    if ((S & 3) == (S >> 2)) return c->wd[S & 3];
    if (S == 9 || S == 6) return c->p.t;
    return 0.0;
}
double orc_vertex_weight(const orc_chain* c, int S) { return vweight(c, S & 15); }

/* heat-bath choice among n weights with one uniform u:
   r = u * sum; first m with W_m > 0 and r < cumulative sum; else the last
   m with W_m > 0. */
static int choose(const double* W, int n, double u)
{
    double tot = 0.0;
    for (int m = 0; m < n; m++) tot = tot + W[m];
    double r = u * tot, cum = 0.0;
    int last = -1;
    for (int m = 0; m < n; m++) {
        cum = cum + W[m];
        if (W[m] > 0.0) {
            last = m;
            if (r < cum) return m;
        }
    }
    return last;
}
int orc_test_choose(const double* w, int n, double u) { return choose(w, n, u); }

/* ------------------------------------------------------------------ */
/* tables                                                              */
/* ------------------------------------------------------------------ */
/* Directed-loop pair weights w_ij = w_ji with row sums w_i
   ("Worm scattering"), minimal-bounce solution over the allowed exits. */
static void solve_pairs(const double w[4], double W[4][4])
{
    memset(W, 0, sizeof(double) * 16);
    int idx[4], n = 0;
    for (int j = 0; j < 4; j++) if (w[j] > 0.0) idx[n++] = j;
    /* stable sort by weight, descending */
    for (int a = 1; a < n; a++) {
        int v = idx[a], b = a - 1;
        while (b >= 0 && w[idx[b]] < w[v]) { idx[b + 1] = idx[b]; b--; }
        idx[b + 1] = v;
    }
    if (n == 0) return;
    if (n == 1) { W[idx[0]][idx[0]] = w[idx[0]]; return; }
    int ja = idx[0], jb = idx[1], jc = (n == 3) ? idx[2] : -1;
    double a = w[ja], b = w[jb], cc = (n == 3) ? w[jc] : 0.0;
    if (a <= b + cc) {
        W[ja][jb] = W[jb][ja] = ((a + b) - cc) * 0.5;
        if (jc >= 0) {
            W[ja][jc] = W[jc][ja] = ((a + cc) - b) * 0.5;
            W[jb][jc] = W[jc][jb] = ((b + cc) - a) * 0.5;
        }
    } else {
        W[ja][ja] = (a - b) - cc;
        W[ja][jb] = W[jb][ja] = b;
        if (jc >= 0) W[ja][jc] = W[jc][ja] = cc;
    }
}

static void build_tables(orc_chain* c)
{
    const orc_params* p = &c->p;
    c->M = 1 << p->ticks_log2;
    c->delta = p->beta / (double)c->M;
    c->lambda = p->eta * c->delta;
    for (int g = 0; g < 4; g++)
        for (int v = 0; v < 256; v++)
            c->F[g][v] = expm1(c->lambda * (double)((uint64_t)v << (8 * g)));

    /* E_b(sa,sc) = V sa sc - (mu/4)(sa+sc): the site term split over the
       four bonds of a site (hard-core Bose-Hubbard model, Eq. (BH)) */
    double Eb[4], Emax = 0.0;
    for (int s = 0; s < 4; s++) {
        int sa = s & 1, sc = s >> 1;
        Eb[s] = p->V * (double)(sa & sc) - (p->mu * 0.25) * (double)(sa + sc);
        if (s == 0 || Eb[s] > Emax) Emax = Eb[s];
    }
    if (isnan(p->C)) c->C = Emax + (p->t > 0.0 ? 0.5 * p->t : 0.5);
    else c->C = p->C;
    c->rho_max = 0.0;
    for (int s = 0; s < 4; s++) {
        c->wd[s] = c->C - Eb[s];
        if (s == 0 || c->wd[s] > c->rho_max) c->rho_max = c->wd[s];
    }
    for (int s = 0; s < 4; s++) c->acc[s] = c->wd[s] / c->rho_max;

    for (int k = 0; k <= c->ntau; k++)
        c->T[k] = (int32_t)(((int64_t)k * (int64_t)c->M) / c->ntau);

    /* Poisson(rho_max * Delta * dT_k) CDF of candidate counts per slab */
    for (int k = 0; k < c->ntau; k++) {
        double* cdf = c->cdf + (size_t)k * KMAX;
        double mu = c->rho_max * (c->delta * (double)(c->T[k + 1] - c->T[k]));
        double pj = exp(-mu), cum = pj;
        int j = 0;
        cdf[0] = cum;
        for (;;) {
            j++;
            pj = (pj * mu) / (double)j;
            if ((double)j > mu && pj < 0x1.0p-64) break;
            if (j >= KMAX - 1) break;
            cum = cum + pj;
            cdf[j] = cum;
        }
        cdf[j] = 2.0;
        c->cdf_len[k] = j + 1;
    }

    /* scattering table: cumulative P(exit j | S0, entry i) = w_ji / w_i */
    for (int S0 = 0; S0 < 16; S0++) {
        double w[4];
        for (int j = 0; j < 4; j++) w[j] = vweight(c, S0 ^ (1 << j));
        double W[4][4];
        solve_pairs(w, W);
        for (int i = 0; i < 4; i++) {
            for (int j = 0; j < 4; j++) c->pairw[S0][i][j] = W[i][j];
            if (!(w[i] > 0.0)) {
                for (int j = 0; j < 4; j++) c->scat[S0][i][j] = 2.0;
                continue;
            }
            int jlast = 0;
            for (int j = 0; j < 4; j++) if (W[j][i] > 0.0) jlast = j;
            double cum = 0.0;
            for (int j = 0; j < 4; j++) {
                cum = cum + W[j][i] / w[i];
                c->scat[S0][i][j] = (j >= jlast) ? 2.0 : cum;
            }
        }
    }

    c->ncycle = p->n_cycle > 0 ? p->n_cycle : (int)ceil(4.0 * c->C / p->eta);
}

/* ------------------------------------------------------------------ */
/* event lists                                                         */
/* ------------------------------------------------------------------ */
static void el_reserve(orc_chain* c, elist* l, int n)
{
    if (n <= l->cap) return;
    int cap = l->cap ? l->cap : 16;
    while (cap < n) cap *= 2;
    ev_t* e = (ev_t*)realloc(l->e, sizeof(ev_t) * (size_t)cap);
    if (!e) { c->flags |= FLAG_NOMEM; return; }
    l->e = e; l->cap = cap;
}
static void el_insert_at(orc_chain* c, elist* l, int pos, ev_t e)
{
    el_reserve(c, l, l->n + 1);
    if (c->flags & FLAG_NOMEM) return;
    memmove(l->e + pos + 1, l->e + pos, sizeof(ev_t) * (size_t)(l->n - pos));
    l->e[pos] = e;
    l->n++;
}
static void el_remove_at(elist* l, int pos)
{
    memmove(l->e + pos, l->e + pos + 1, sizeof(ev_t) * (size_t)(l->n - pos - 1));
    l->n--;
}
/* sort key comparison: (tick, class, bond id); returns <0, 0, >0 */
static int key_cmp(const orc_chain* c, int site, const ev_t* e,
                   int32_t tick, int cls, int64_t bid)
{
    if (e->tick != tick) return e->tick < tick ? -1 : 1;
    if (e->worm != cls) return e->worm < cls ? -1 : 1;
    if (e->worm) return 0;
    int64_t eb = bond_id(c, site, e->dir);
    if (eb != bid) return eb < bid ? -1 : 1;
    return 0;
}
/* position where an object with key (tick, cls, bid) goes */
static int el_lower_bound(const orc_chain* c, int site, int32_t tick, int cls, int64_t bid)
{
    const elist* l = &c->site[site];
    int i = 0;
    while (i < l->n && key_cmp(c, site, &l->e[i], tick, cls, bid) < 0) i++;
    return i;
}
static int el_insert_sorted(orc_chain* c, int site, ev_t e)
{
    int64_t bid = e.worm ? 0 : bond_id(c, site, e.dir);
    int pos = el_lower_bound(c, site, e.tick, e.worm, bid);
    el_insert_at(c, &c->site[site], pos, e);
    return pos;
}
static int find_worm(const orc_chain* c, int site, int32_t slot)
{
    const elist* l = &c->site[site];
    for (int i = 0; i < l->n; i++)
        if (l->e[i].worm && l->e[i].tick == slot) return i;
    return -1;
}
static int find_vertex(const orc_chain* c, int site, int32_t tick, int dir)
{
    const elist* l = &c->site[site];
    for (int i = 0; i < l->n; i++)
        if (!l->e[i].worm && l->e[i].tick == tick && l->e[i].dir == dir) return i;
    return -1;
}
/* index range [*lo, *hi) of the events of `site` in slab k */
static void slab_range(const orc_chain* c, int site, int k, int* lo, int* hi)
{
    const elist* l = &c->site[site];
    int i = 0;
    while (i < l->n && l->e[i].tick < c->T[k]) i++;
    *lo = i;
    while (i < l->n && l->e[i].tick < c->T[k + 1]) i++;
    *hi = i;
}
/* occupation just below event index i (which lies in slab k) */
static int state_below(const orc_chain* c, int site, int k, int i)
{
    const elist* l = &c->site[site];
    if (i > 0 && l->e[i - 1].tick >= c->T[k]) return l->e[i - 1].up;
    return c->bstate[(size_t)k * c->N + site];
}

/* ------------------------------------------------------------------ */
/* worm law on one interval (Eq. (worm), hard-core form)               */
/* ------------------------------------------------------------------ */
#define NWMAX 4096
/* Draw the worms of an interval of `ell` free slots whose end states
   differ by parity sigma: the count n ~ x^n / n! / f_sigma(x),
   x = eta*Delta*ell, n = sigma mod 2, n <= ell, by inversion; then n
   distinct uniform slots (offsets in [0, ell)), sorted; then one direction
   bit per worm in ascending slot order.  Returns n. */
static int sample_worms(orc_chain* c, rstream* s, int64_t ell, int sigma,
                        int32_t* off, uint8_t* dirs)
{
    if (ell == 0) {
        if (sigma) c->flags |= FLAG_SIGMA;
        return 0;
    }
    double f = fleg(c, sigma, ell);
    double x = c->lambda * (double)ell;
    double xx = x * x;
    int64_t nmax = ell < NWMAX ? ell : NWMAX;
    int n = -1;
    for (int tries = 0; tries < 1000; tries++) {
        double U = u53(rs_next(s)) * f;
        int64_t k = sigma;
        double T = sigma ? x : 1.0;
        double S = T;
        while (!(U < S) && k + 2 <= nmax) {
            T = (T * xx) / (double)((k + 1) * (k + 2));
            k += 2;
            S = S + T;
        }
        if (U < S && k <= nmax) { n = (int)k; break; }
    }
    if (n < 0) { c->flags |= FLAG_REDRAW; return 0; }
    for (int i = 0; i < n; i++) {
        int32_t r;
        int again, guard = 0;
        do {
            r = (int32_t)below(rs_next(s), (uint64_t)ell);
            again = 0;
            for (int j = 0; j < i; j++) if (off[j] == r) { again = 1; break; }
        } while (again && ++guard < 100000);
        if (again) { c->flags |= FLAG_REDRAW; return 0; }
        off[i] = r;
    }
    for (int a = 1; a < n; a++) {            /* insertion sort */
        int32_t v = off[a]; int b = a - 1;
        while (b >= 0 && off[b] > v) { off[b + 1] = off[b]; b--; }
        off[b + 1] = v;
    }
    for (int i = 0; i < n; i++) dirs[i] = (uint8_t)(rs_next(s) >> 63);
    return n;
}

/* insert the worms of an interval starting at slot `base` on `site`,
   with occupation `p` just above the lower end */
static void place_worms(orc_chain* c, rstream* s, int site, int32_t base,
                        int64_t ell, int sigma, int p)
{
    static int32_t off[NWMAX];
    static uint8_t dirs[NWMAX];
    int n = sample_worms(c, s, ell, sigma, off, dirs);
    int st = p;
    for (int i = 0; i < n; i++) {
        st ^= 1;
        ev_t e = { base + off[i], 1, dirs[i], (uint8_t)st };
        el_insert_sorted(c, site, e);
    }
}

int orc_test_worms(orc_chain* c, uint32_t phase, uint32_t unit, int32_t ell,
                   int sigma, int32_t* offsets, uint8_t* dirs, int cap)
{
    static int32_t off[NWMAX];
    static uint8_t d[NWMAX];
    rstream s; rs_init(&s, c, phase, unit);
    int n = sample_worms(c, &s, ell, sigma, off, d);
    for (int i = 0; i < n && i < cap; i++) { offsets[i] = off[i]; dirs[i] = d[i]; }
    return n;
}

/* ------------------------------------------------------------------ */
/* Step 3: vertex phase                                                */
/* ------------------------------------------------------------------ */
/* occupation of `site` seen by an object with key (tick, vertex, bid) in
   slab k: just above the last event ordering before it */
static int state_seen(const orc_chain* c, int site, int k, int32_t tick, int64_t bid)
{
    const elist* l = &c->site[site];
    int lo, hi;
    slab_range(c, site, k, &lo, &hi);
    int s = c->bstate[(size_t)k * c->N + site];
    for (int i = lo; i < hi; i++) {
        if (key_cmp(c, site, &l->e[i], tick, 0, bid) < 0) s = l->e[i].up;
        else break;
    }
    return s;
}

static int32_t pos2(const ev_t* e) { return 2 * e->tick + (e->worm ? 1 : 0); }

/* integral of n_a n_c over slab k in half-ticks, on the current state */
static int64_t bond_nn(const orc_chain* c, int a, int cc, int k)
{
    const elist* la = &c->site[a];
    const elist* lc = &c->site[cc];
    int ia, ha, ic, hc;
    slab_range(c, a, k, &ia, &ha);
    slab_range(c, cc, k, &ic, &hc);
    int sa = c->bstate[(size_t)k * c->N + a];
    int sc = c->bstate[(size_t)k * c->N + cc];
    int64_t last = 2 * (int64_t)c->T[k], acc = 0;
    while (ia < ha || ic < hc) {
        int takea;
        if (ia >= ha) takea = 0;
        else if (ic >= hc) takea = 1;
        else takea = pos2(&la->e[ia]) <= pos2(&lc->e[ic]);
        const ev_t* e = takea ? &la->e[ia++] : &lc->e[ic++];
        int64_t pos = pos2(e);
        acc += (int64_t)(sa & sc) * (pos - last);
        last = pos;
        if (takea) sa = e->up; else sc = e->up;
    }
    acc += (int64_t)(sa & sc) * (2 * (int64_t)c->T[k + 1] - last);
    return acc;
}

static void vertex_phase(orc_chain* c)
{
    int32_t cand[KMAX + 8], kinks[4096];
    for (int64_t b = 0; b < 2 * (int64_t)c->N; b++) {
        int a = (int)(b >> 1), d = (int)(b & 1), cc = nb(c, a, d);
        vlist* out = &c->bondv[b];
        out->n = 0;
        for (int k = 0; k < c->ntau; k++) {
            c->cur.nn2 += bond_nn(c, a, cc, k);
            /* kinks of this bond in slab k survive */
            int lo, hi, nk = 0;
            slab_range(c, a, k, &lo, &hi);
            for (int i = lo; i < hi; i++) {
                const ev_t* e = &c->site[a].e[i];
                if (!e->worm && e->dir == d && e->up != state_below(c, a, k, i)) {
                    if (nk < 4096) kinks[nk++] = e->tick;
                    else c->flags |= FLAG_REDRAW;
                }
            }
            rstream s;
            rs_init(&s, c, RNG_V, (uint32_t)(b * c->ntau + k));
            /* candidate count: Poisson(rho_max * Delta * dT_k), inversion */
            const double* cdf = c->cdf + (size_t)k * KMAX;
            double u = u53(rs_next(&s));
            int n = 0;
            while (!(u < cdf[n])) n++;
            int64_t dT = c->T[k + 1] - c->T[k];
            for (int i = 0; i < n; i++) {
                int32_t tau;
                int again, guard = 0;
                do {
                    tau = c->T[k] + (int32_t)below(rs_next(&s), (uint64_t)dT);
                    again = 0;
                    for (int j = 0; j < nk; j++) if (kinks[j] == tau) again = 1;
                    for (int j = 0; j < i; j++) if (cand[j] == tau) again = 1;
                } while (again && ++guard < 100000);
                if (again) { c->flags |= FLAG_REDRAW; n = i; break; }
                cand[i] = tau;
            }
            for (int x = 1; x < n; x++) {
                int32_t v = cand[x]; int y = x - 1;
                while (y >= 0 && cand[y] > v) { cand[y + 1] = cand[y]; y--; }
                cand[y + 1] = v;
            }
            /* thinning: accept with w_d(state)/rho_max (density proportional
               to the diagonal matrix element, Step 3) */
            for (int i = 0; i < n; i++) {
                int sa = state_seen(c, a, k, cand[i], b);
                int sc = state_seen(c, cc, k, cand[i], b);
                double uu = u53(rs_next(&s));
                if (uu < c->acc[sa | (sc << 1)]) {
                    if (out->n == out->cap) {
                        int cap = out->cap ? 2 * out->cap : 16;
                        newv_t* v = (newv_t*)realloc(out->v, sizeof(newv_t) * (size_t)cap);
                        if (!v) { c->flags |= FLAG_NOMEM; return; }
                        out->v = v; out->cap = cap;
                    }
                    newv_t nv = { cand[i], (uint8_t)sa, (uint8_t)sc };
                    out->v[out->n++] = nv;
                }
            }
        }
    }
}

/* ------------------------------------------------------------------ */
/* Step 4: erase all worms, regenerate them on every interval          */
/* ------------------------------------------------------------------ */
typedef struct { int32_t tick; int64_t bid; uint8_t dir, below, above; } rv_t;

static int rv_cmp(const void* x, const void* y)
{
    const rv_t* a = (const rv_t*)x; const rv_t* b = (const rv_t*)y;
    if (a->tick != b->tick) return a->tick < b->tick ? -1 : 1;
    if (a->bid != b->bid) return a->bid < b->bid ? -1 : 1;
    return 0;
}

static void worm_phase_R(orc_chain* c)
{
    rv_t* vs = NULL; int vcap = 0;
    elist fresh = { NULL, 0, 0 };
    for (int i = 0; i < c->N; i++) {
        fresh.n = 0;
        for (int k = 0; k < c->ntau; k++) {
            int nv = 0;
            int lo, hi;
            slab_range(c, i, k, &lo, &hi);
            /* kinks of this site survive with their roots */
            int need = (hi - lo) + 16;
            const int nbr[4] = { i, i, nb(c, i, 2), nb(c, i, 3) };
            for (int d = 0; d < 4; d++)
                need += c->bondv[2 * (int64_t)nbr[d] + (d & 1)].n;
            if (need > vcap) {
                vcap = 2 * need;
                rv_t* nvs = (rv_t*)realloc(vs, sizeof(rv_t) * (size_t)vcap);
                if (!nvs) { c->flags |= FLAG_NOMEM; free(vs); free(fresh.e); return; }
                vs = nvs;
            }
            for (int j = lo; j < hi; j++) {
                const ev_t* e = &c->site[i].e[j];
                if (e->worm) continue;
                int below_s = state_below(c, i, k, j);
                if (e->up == below_s) continue;        /* diagonal: erased */
                rv_t r = { e->tick, bond_id(c, i, e->dir), e->dir,
                           (uint8_t)below_s, e->up };
                vs[nv++] = r;
            }
            /* new diagonal vertices of the four bonds of site i */
            for (int d = 0; d < 4; d++) {
                int64_t b = 2 * (int64_t)nbr[d] + (d & 1);
                const vlist* bl = &c->bondv[b];
                for (int j = 0; j < bl->n; j++) {
                    const newv_t* v = &bl->v[j];
                    if (v->tick < c->T[k] || v->tick >= c->T[k + 1]) continue;
                    uint8_t s = d < 2 ? v->sa : v->sc;
                    rv_t r = { v->tick, b, (uint8_t)d, s, s };
                    vs[nv++] = r;
                }
            }
            qsort(vs, (size_t)nv, sizeof(rv_t), rv_cmp);

            rstream s;
            rs_init(&s, c, RNG_R, (uint32_t)((int64_t)i * c->ntau + k));
            int32_t lo_tick = c->T[k];
            int p = c->bstate[(size_t)k * c->N + i];
            static int32_t off[NWMAX];
            static uint8_t dirs[NWMAX];
            for (int j = 0; j <= nv; j++) {
                int32_t hi_tick; int q;
                if (j < nv) { hi_tick = vs[j].tick; q = vs[j].below; }
                else { hi_tick = c->T[k + 1]; q = c->bstate[(size_t)((k + 1) % c->ntau) * c->N + i]; }
                /* interval j (j-th gap between the slab's vertices, from the
                   bottom) draws from word 2^17 j of the (site, slab) stream */
                s.w = (uint64_t)j << 17;
                s.have = 0;
                int n = sample_worms(c, &s, (int64_t)hi_tick - lo_tick, p ^ q, off, dirs);
                el_reserve(c, &fresh, fresh.n + n + 1);
                if (c->flags & FLAG_NOMEM) { free(vs); free(fresh.e); return; }
                int st = p;
                for (int w = 0; w < n; w++) {
                    st ^= 1;
                    ev_t e = { lo_tick + off[w], 1, dirs[w], (uint8_t)st };
                    fresh.e[fresh.n++] = e;
                }
                if (j < nv) {
                    ev_t e = { vs[j].tick, 0, vs[j].dir, vs[j].above };
                    fresh.e[fresh.n++] = e;
                    lo_tick = vs[j].tick;
                    p = vs[j].above;
                }
            }
        }
        /* swap the new list in */
        elist* l = &c->site[i];
        el_reserve(c, l, fresh.n);
        if (c->flags & FLAG_NOMEM) break;
        memcpy(l->e, fresh.e, sizeof(ev_t) * (size_t)fresh.n);
        l->n = fresh.n;
    }
    free(vs);
    free(fresh.e);
}

/* ------------------------------------------------------------------ */
/* Steps 5-6: worm scattering, N_cycle times, per domain               */
/* ------------------------------------------------------------------ */
/* lower end of the free slots above object index j of `site` in slab k
   (j < lo of slab: the boundary T_k) */
static int32_t lofirst(const orc_chain* c, int site, int k, int j)
{
    const elist* l = &c->site[site];
    if (j >= 0 && l->e[j].tick >= c->T[k]) return l->e[j].tick + (l->e[j].worm ? 1 : 0);
    return c->T[k];
}
/* exclusive upper end of the free slots below object index j */
static int32_t hiexcl(const orc_chain* c, int site, int k, int j)
{
    const elist* l = &c->site[site];
    if (j < l->n && l->e[j].tick < c->T[k + 1]) return l->e[j].tick;
    return c->T[k + 1];
}

/* one attempt of one worm (Step 5); returns 0 */
static void worm_step(orc_chain* c, int k, wref* w, rstream* s)
{
    /* every attempt draws three words, used or not: the enter test, the
       exit leg and the landing slot */
    uint64_t w_enter = rs_next(s), w_exit = rs_next(s), w_slot = rs_next(s);
    int x = w->site;
    int iw = find_worm(c, x, w->slot);
    if (iw < 0) { c->flags |= FLAG_STATE; return; }
    elist* lx = &c->site[x];
    int up = lx->e[iw].dir;
    int ia = up ? iw + 1 : iw - 1;
    int blocked = 0;
    if (up) blocked = !(ia < lx->n && lx->e[ia].tick < c->T[k + 1]);
    else blocked = !(ia >= 0 && lx->e[ia].tick >= c->T[k]);
    if (!blocked && lx->e[ia].worm) blocked = 1;           /* worm ahead */
    int d = 0, a = 0, cc = 0;
    if (!blocked) {
        d = lx->e[ia].dir;
        a = d < 2 ? x : nb(c, x, d);
        if (is_cross(c, a, d & 1)) blocked = 1;           /* spatial boundary */
    }
    if (blocked) { lx->e[iw].dir ^= 1; return; }

    int bd = d & 1;
    cc = nb(c, a, bd);
    int32_t t = lx->e[ia].tick;
    int va = (x == a) ? ia : find_vertex(c, a, t, bd);
    int vc = (x == cc) ? ia : find_vertex(c, cc, t, bd + 2);
    if (va < 0 || vc < 0) { c->flags |= FLAG_STATE; return; }
    /* leg lengths, the moving worm excluded (it would be adjacent) */
    int64_t L[4];
    {
        int j;
        j = va - 1; if (x == a && j == iw) j--;  L[0] = t - lofirst(c, a, k, j);
        j = vc - 1; if (x == cc && j == iw) j--; L[1] = t - lofirst(c, cc, k, j);
        j = va + 1; if (x == a && j == iw) j++;  L[2] = hiexcl(c, a, k, j) - t;
        j = vc + 1; if (x == cc && j == iw) j++; L[3] = hiexcl(c, cc, k, j) - t;
    }
    int i = up ? (x == a ? 0 : 1) : (x == a ? 2 : 3);
    int64_t Lmin = L[0];
    for (int j = 1; j < 4; j++) if (L[j] < Lmin) Lmin = L[j];
    /* enter with probability L_min / L_i */
    uint64_t r = below(w_enter, (uint64_t)L[i]);
    if ((int64_t)r >= Lmin) { lx->e[iw].dir ^= 1; return; }

    int S = state_below(c, a, k, va) | (state_below(c, cc, k, vc) << 1)
          | (c->site[a].e[va].up << 2) | (c->site[cc].e[vc].up << 3);
    int S0 = S ^ (1 << i);
    double u = u53(w_exit);
    int j = 0;
    while (!(u < c->scat[S0][i][j])) j++;
    uint64_t r2 = below(w_slot, (uint64_t)L[j]);

    /* move: remove the worm from leg i */
    int wup = lx->e[iw].up;
    if (i >= 2) {                      /* worm was above the vertex end on x */
        int vx = (x == a) ? va : vc;
        lx->e[vx].up = (uint8_t)wup;
    }
    el_remove_at(lx, iw);
    /* insert it on leg j */
    int y = (j & 1) ? cc : a;
    int vy = find_vertex(c, y, t, (j & 1) ? bd + 2 : bd);
    if (vy < 0) { c->flags |= FLAG_STATE; return; }
    int32_t slot = (j >= 2) ? t + (int32_t)r2 : t - 1 - (int32_t)r2;
    ev_t e = { slot, 1, (uint8_t)(j >= 2 ? 1 : 0), 0 };
    if (j >= 2) {
        e.up = c->site[y].e[vy].up;
        c->site[y].e[vy].up ^= 1;
        el_insert_sorted(c, y, e);
    } else {
        int pos = el_insert_sorted(c, y, e);
        c->site[y].e[pos].up = (uint8_t)(state_below(c, y, k, pos) ^ 1);
    }
    w->site = y;
    w->slot = slot;
}

static void measure_site(orc_chain* c, int i)
{
    for (int k = 0; k < c->ntau; k++) {
        int lo, hi;
        slab_range(c, i, k, &lo, &hi);
        const elist* l = &c->site[i];
        int st = c->bstate[(size_t)k * c->N + i];
        int64_t last = 2 * (int64_t)c->T[k];
        int32_t ilo = c->T[k];         /* lower end of the current interval */
        int par = 0;                   /* worm parity in it                 */
        for (int j = lo; j <= hi; j++) {
            int64_t pos = (j < hi) ? pos2(&l->e[j]) : 2 * (int64_t)c->T[k + 1];
            c->cur.occ2 += (int64_t)st * (pos - last);
            last = pos;
            if (j < hi && l->e[j].worm) {
                c->cur.nw++;
                par ^= 1;
                st = l->e[j].up;
                continue;
            }
            /* an interval ends at a vertex or at the slab top */
            int32_t ihi = (j < hi) ? l->e[j].tick : c->T[k + 1];
            int64_t ell = (int64_t)ihi - ilo;
            if (ell > 0) {
                double th = tanh_ell(c, ell);
                double g = par ? 1.0 / th : th;
                c->cur.qimp += (double)ell * g;
            }
            if (j < hi) {
                const ev_t* e = &l->e[j];
                if (e->dir < 2) {
                    c->cur.nv++;
                    if (e->up != st) c->cur.nkink++;
                }
                st = e->up;
                ilo = e->tick;
                par = 0;
            }
        }
    }
}

/* ------------------------------------------------------------------ */
/* Green function of Q = b + b^+ (Supplemental S-I, n = 2)             */
/* ------------------------------------------------------------------ */
/* rho(X)/eta on the interval holding X: tanh(lambda l) for an even number
   of worms in it, coth(lambda l) for an odd number (the ratio of the
   hard-core propagators f split at X; it does not depend on where X lies in
   the interval).  Intervals are delimited by vertices and the temporal
   domain boundaries.  Two points on different intervals give the product of
   their ratios (the product rule of S-I).  Two points on the same interval
   (same site): the split ratio is eta^2 <q|e^{l3 eta Q} Q e^{l2 eta Q} Q
   e^{l1 eta Q}|p> / <q|e^{l eta Q}|p> = eta^2, because Q commutes with
   e^{x Q} and Q^2 = 1, so the sample is 1. */
typedef struct { int32_t lo, hi; double g; } gint_t;

/* the intervals of `site` over [0, M), in time order; returns their count */
static int green_intervals(const orc_chain* c, int site, gint_t* out)
{
    const elist* l = &c->site[site];
    int n = 0;
    for (int k = 0; k < c->ntau; k++) {
        int lo, hi;
        slab_range(c, site, k, &lo, &hi);
        int32_t start = c->T[k];
        int par = 0;
        for (int j = lo; j <= hi; j++) {
            if (j < hi && l->e[j].worm) { par ^= 1; continue; }
            int32_t end = (j < hi) ? l->e[j].tick : c->T[k + 1];
            int64_t ell = (int64_t)end - start;
            if (ell > 0) {
                double th = tanh_ell(c, ell);
                out[n].lo = start; out[n].hi = end; out[n].g = par ? 1.0 / th : th;
                n++;
            }
            start = end;
            par = 0;
        }
    }
    return n;
}

/* G(r, dt) = (1/N) sum_i <Q_i(tau) Q_{i+r}(tau + dt)>, averaged over tau in
   [0, beta): on the current configuration,
   (1 / (M N)) sum_i int_0^M h_i(tau) dtau with h the two-point sample of the
   points (i, tau) and (i + r, tau + dt mod M).  disp holds (rx, ry, dt)
   triples; dt in ticks. */
int orc_green(const orc_chain* c, const int32_t* disp, int n, double* out)
{
    if (n < 0 || (n > 0 && (!disp || !out))) return ORC_EINVAL;
    int cap = 0;
    for (int i = 0; i < c->N; i++) if (c->site[i].n + c->ntau > cap) cap = c->site[i].n + c->ntau;
    gint_t* A = (gint_t*)malloc(sizeof(gint_t) * (size_t)(cap + 1));
    gint_t* B = (gint_t*)malloc(sizeof(gint_t) * (size_t)(cap + 1));
    if (!A || !B) { free(A); free(B); return ORC_ENOMEM; }
    for (int d = 0; d < n; d++) {
        int rx = ((disp[3 * d] % c->Lx) + c->Lx) % c->Lx;
        int ry = ((disp[3 * d + 1] % c->Ly) + c->Ly) % c->Ly;
        int32_t dt = (int32_t)((((int64_t)disp[3 * d + 2] % c->M) + c->M) % c->M);
        double sum = 0.0;
        for (int i = 0; i < c->N; i++) {
            int x = i % c->Lx, y = i / c->Lx;
            int jj = ((y + ry) % c->Ly) * c->Lx + (x + rx) % c->Lx;
            int na = green_intervals(c, i, A);
            int nb = green_intervals(c, jj, B);
            /* b: the interval of jj holding time dt (the partner of tau = 0) */
            int b = 0;
            while (B[b].hi <= dt) b++;
            int32_t pos = dt;              /* partner time of tau */
            int32_t tau = 0;
            int a = 0;
            while (tau < c->M && a < na) {
                int32_t len = A[a].hi - tau;
                int32_t lenb = B[b].hi - pos;
                if (lenb < len) len = lenb;
                double h = (jj == i && a == b) ? 1.0 : A[a].g * B[b].g;
                sum += (double)len * h;
                tau += len;
                pos += len;
                if (tau == A[a].hi) a++;
                if (pos == B[b].hi) {
                    b++;
                    if (b == nb) { b = 0; pos = 0; }
                }
            }
        }
        out[d] = sum / ((double)c->M * (double)c->N);
    }
    free(A);
    free(B);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* n-point functions of b, b^+ and Q (Supplemental S-I, general n)     */
/* ------------------------------------------------------------------ */
/* The configuration's weight is a product over intervals (delimited by
   vertices and temporal domain boundaries) of <q| exp(l eta Delta Q) |p>,
   p and q the occupations just above its lower and just below its upper
   end: the worms inside an interval are summed over.  An operator inserted
   at a point of an interval multiplies that factor by
     <q| E(l_top) O_m E(..) ... O_1 E(l_bottom) |p> / <q| E(l) |p>,
   E(l) = exp(l eta Delta Q), the operators in time order; points on
   different intervals give the product of their intervals' factors.  A
   point at tick t sits at t + 1/4: between a vertex at t and the worm slot
   t + 1/2, so l_bottom = t - lo slots lie below it and hi - t above. */
enum { ORC_OP_Q = 0, ORC_OP_B = 1, ORC_OP_BD = 2 };

typedef struct { int site; int32_t t; int op, idx; int32_t lo, hi; int p, q, grp; } cpt_t;

/* interval of `site` holding time t + 1/4: its ends lo <= t < hi, the
   occupation p just above lo and q just below hi */
static void point_interval(const orc_chain* c, int site, int32_t t, int32_t* lo, int32_t* hi, int* p, int* q)
{
    int k = slab_of(c, t);
    const elist* l = &c->site[site];
    int a, b;
    slab_range(c, site, k, &a, &b);
    *lo = c->T[k];
    *p = c->bstate[(size_t)k * c->N + site];
    *hi = c->T[k + 1];
    *q = c->bstate[(size_t)((k + 1) % c->ntau) * c->N + site];
    for (int j = a; j < b; j++) {
        const ev_t* e = &l->e[j];
        if (e->worm) continue;
        if (e->tick <= t) { *lo = e->tick; *p = e->up; }
        else { *hi = e->tick; *q = state_below(c, site, k, j); break; }
    }
}

/* v <- E(ell) v with E = [[cosh, sinh], [sinh, cosh]](lambda ell) */
static void prop2(const orc_chain* c, int64_t ell, double v[2])
{
    double ch = fleg(c, 0, ell), sh = fleg(c, 1, ell);
    double n0 = ch * v[0] + sh * v[1];
    double n1 = sh * v[0] + ch * v[1];
    v[0] = n0; v[1] = n1;
}
static void apply_op(int op, double v[2])
{
    double a = v[0], b = v[1];
    if (op == ORC_OP_Q) { v[0] = b; v[1] = a; }
    else if (op == ORC_OP_B) { v[0] = b; v[1] = 0.0; }     /* b|1> = |0> */
    else { v[0] = 0.0; v[1] = a; }                        /* b^+|0> = |1> */
}

/* one sample: points (site_k, t_k) of one base point, in the order listed */
static double corr_sample(const orc_chain* c, cpt_t* P, int np)
{
    for (int k = 0; k < np; k++) {
        point_interval(c, P[k].site, P[k].t, &P[k].lo, &P[k].hi, &P[k].p, &P[k].q);
        P[k].grp = -1;
    }
    double prod = 1.0;
    for (int k = 0; k < np; k++) {
        if (P[k].grp >= 0) continue;
        /* the group of point k: every point on the same interval */
        int mem[16], nm = 0;
        for (int m = k; m < np; m++)
            if (P[m].site == P[k].site && P[m].lo == P[k].lo && P[m].hi == P[k].hi) {
                P[m].grp = k;
                mem[nm++] = m;
            }
        /* bottom to top: ascending time; at equal times the later-listed
           point acts first (the first listed is leftmost) */
        for (int a = 1; a < nm; a++) {
            int v = mem[a], b = a - 1;
            while (b >= 0 && (P[mem[b]].t > P[v].t || (P[mem[b]].t == P[v].t && mem[b] < v))) {
                mem[b + 1] = mem[b]; b--;
            }
            mem[b + 1] = v;
        }
        double v[2] = { 0.0, 0.0 };
        v[P[k].p] = 1.0;
        int32_t cur = P[k].lo;
        for (int a = 0; a < nm; a++) {
            prop2(c, (int64_t)P[mem[a]].t - cur, v);
            apply_op(P[mem[a]].op, v);
            cur = P[mem[a]].t;
        }
        prop2(c, (int64_t)P[k].hi - cur, v);
        double den = fleg(c, P[k].p ^ P[k].q, (int64_t)P[k].hi - P[k].lo);
        prod = prod * (v[P[k].q] / den);
    }
    return prod;
}

int orc_correlator(const orc_chain* c, int npt, const int32_t* pts, int ncorr, int nbase, double* out)
{
    if (npt < 1 || npt > 16 || ncorr < 1 || nbase < 1 || !pts || !out) return ORC_EINVAL;
    for (int i = 0; i < npt * ncorr; i++)
        if (pts[4 * i + 3] < 0 || pts[4 * i + 3] > 2) return ORC_EINVAL;
    cpt_t P[16];
    for (int cc = 0; cc < ncorr; cc++) {
        const int32_t* q = pts + (size_t)4 * npt * cc;
        double sum = 0.0;
        for (int i = 0; i < c->N; i++) {
            int x = i % c->Lx, y = i / c->Lx;
            for (int j = 0; j < nbase; j++) {
                int64_t tau = ((int64_t)j * c->M) / nbase;
                for (int k = 0; k < npt; k++) {
                    int rx = ((q[4 * k] % c->Lx) + c->Lx) % c->Lx;
                    int ry = ((q[4 * k + 1] % c->Ly) + c->Ly) % c->Ly;
                    P[k].site = ((y + ry) % c->Ly) * c->Lx + (x + rx) % c->Lx;
                    P[k].t = (int32_t)((((tau + (int64_t)q[4 * k + 2]) % c->M) + c->M) % c->M);
                    P[k].op = q[4 * k + 3];
                    P[k].idx = k;
                }
                sum += corr_sample(c, P, npt);
            }
        }
        out[cc] = sum / ((double)c->N * (double)nbase);
    }
    return ORC_OK;
}

static void scatter_phase(orc_chain* c)
{
    int ndsp = c->p.dom_x * c->p.dom_y;
    wref* list = NULL; int lcap = 0;
    for (int k = 0; k < c->ntau; k++)
    for (int dy = 0; dy < c->p.dom_y; dy++)
    for (int dx = 0; dx < c->p.dom_x; dx++) {
        int D = (k * c->p.dom_y + dy) * c->p.dom_x + dx;
        (void)ndsp;
        /* worm list in (site, slot) order, fixed for the whole phase */
        int nwl = 0;
        for (int ly = 0; ly < c->ey; ly++)
        for (int lx = 0; lx < c->ex; lx++) {
            int site = (dy * c->ey + ly) * c->Lx + dx * c->ex + lx;
            int lo, hi;
            slab_range(c, site, k, &lo, &hi);
            for (int j = lo; j < hi; j++) {
                if (!c->site[site].e[j].worm) continue;
                if (nwl == lcap) {
                    lcap = lcap ? 2 * lcap : 64;
                    wref* nl = (wref*)realloc(list, sizeof(wref) * (size_t)lcap);
                    if (!nl) { c->flags |= FLAG_NOMEM; free(list); return; }
                    list = nl;
                }
                wref r = { site, c->site[site].e[j].tick };
                list[nwl++] = r;
            }
        }
        rstream s;
        rs_init(&s, c, RNG_S, (uint32_t)D);
        for (int cyc = 0; cyc < c->ncycle; cyc++)
            for (int w = 0; w < nwl; w++) worm_step(c, k, &list[w], &s);
    }
    free(list);
    for (int i = 0; i < c->N; i++) measure_site(c, i);
}

/* ------------------------------------------------------------------ */
/* Step 1: temporal-boundary update, Eq. (Para)                        */
/* ------------------------------------------------------------------ */
static void erase_worms(orc_chain* c, int site, int32_t slot_lo, int32_t slot_hi)
{
    elist* l = &c->site[site];
    int j = 0;
    while (j < l->n) {
        if (l->e[j].worm && l->e[j].tick >= slot_lo && l->e[j].tick < slot_hi)
            el_remove_at(l, j);
        else j++;
    }
}
static int site_has_vertex(const orc_chain* c, int site)
{
    const elist* l = &c->site[site];
    for (int j = 0; j < l->n; j++) if (!l->e[j].worm) return 1;
    return 0;
}

static void temporal_phase(orc_chain* c)
{
    int nt = c->ntau;
    for (int i = 0; i < c->N; i++)
    for (int k = 0; k < nt; k++) {
        rstream s;
        rs_init(&s, c, RNG_BT, (uint32_t)((int64_t)i * nt + k));
        uint8_t* sk = &c->bstate[(size_t)k * c->N + i];
        if (nt == 1 && !site_has_vertex(c, i)) {
            /* the whole circle is one interval through the boundary:
               both states carry the same weight cosh(eta*beta) */
            double W[2] = { 1.0, 1.0 };
            int sp = choose(W, 2, u53(rs_next(&s)));
            erase_worms(c, i, 0, c->M);
            place_worms(c, &s, i, 0, c->M, 0, sp);
            *sk = (uint8_t)sp;
            continue;
        }
        const elist* l = &c->site[i];
        int lo, hi;
        /* I_1: from the boundary up to the first vertex of slab k */
        slab_range(c, i, k, &lo, &hi);
        int32_t t1 = c->T[k + 1];
        int q = c->bstate[(size_t)((k + 1) % nt) * c->N + i];
        for (int j = lo; j < hi; j++)
            if (!l->e[j].worm) { t1 = l->e[j].tick; q = state_below(c, i, k, j); break; }
        int64_t l1 = (int64_t)t1 - c->T[k];
        /* I_2: from the last vertex of slab k-1 up to the boundary */
        int kp = (k + nt - 1) % nt;
        int32_t top = c->T[kp + 1];
        slab_range(c, i, kp, &lo, &hi);
        int32_t t2 = c->T[kp];
        int p = c->bstate[(size_t)kp * c->N + i];
        for (int j = hi - 1; j >= lo; j--)
            if (!l->e[j].worm) { t2 = l->e[j].tick; p = l->e[j].up; break; }
        int64_t l2 = (int64_t)top - t2;
        /* P(s') = f_{q s'}(I_1) f_{s' p}(I_2) / f_{qp}(I) */
        double W[2];
        for (int sp = 0; sp < 2; sp++)
            W[sp] = fleg(c, sp ^ q, l1) * fleg(c, p ^ sp, l2);
        int sp = choose(W, 2, u53(rs_next(&s)));
        erase_worms(c, i, c->T[k], t1);
        erase_worms(c, i, t2, top);
        place_worms(c, &s, i, c->T[k], l1, sp ^ q, sp);
        place_worms(c, &s, i, t2, l2, p ^ sp, p);
        *sk = (uint8_t)sp;
    }
}

double orc_test_temporal_p0(const orc_chain* c, int p, int q, int64_t l1, int64_t l2)
{
    double W[2];
    for (int sp = 0; sp < 2; sp++) W[sp] = fleg(c, sp ^ q, l1) * fleg(c, p ^ sp, l2);
    return W[0] / (W[0] + W[1]);
}

/* ------------------------------------------------------------------ */
/* Step 2: spatial-boundary vertex update, Eq. (ParaSpace)             */
/* ------------------------------------------------------------------ */
/* lower delimiter of the leg below event j (a vertex) on `site`, slab k,
   worms ignored: returns its first free slot and the occupation above it */
static void leg_below(const orc_chain* c, int site, int k, int j, int32_t* lo, int* p)
{
    const elist* l = &c->site[site];
    for (int m = j - 1; m >= 0 && l->e[m].tick >= c->T[k]; m--)
        if (!l->e[m].worm) { *lo = l->e[m].tick; *p = l->e[m].up; return; }
    *lo = c->T[k];
    *p = c->bstate[(size_t)k * c->N + site];
}
/* upper delimiter of the leg above event j, worms ignored: its tick and
   the occupation just below it (its root) */
static void leg_above(const orc_chain* c, int site, int k, int j, int32_t* hi, int* q)
{
    const elist* l = &c->site[site];
    for (int m = j + 1; m < l->n && l->e[m].tick < c->T[k + 1]; m++)
        if (!l->e[m].worm) { *hi = l->e[m].tick; *q = state_below(c, site, k, m); return; }
    *hi = c->T[k + 1];
    *q = c->bstate[(size_t)((k + 1) % c->ntau) * c->N + site];
}

static const int ALLOWED[6] = { 0, 5, 6, 9, 10, 15 };

static void spatial_phase(orc_chain* c, int d)
{
    for (int a = 0; a < c->N; a++) {
        if (!is_cross(c, a, d)) continue;
        int cc = nb(c, a, d);
        int64_t b = 2 * (int64_t)a + d;
        int kcur = -1, v = 0;
        int32_t tcur = -1;
        for (;;) {
            /* next vertex of this bond in tick order */
            const elist* la = &c->site[a];
            int32_t t = -1;
            for (int j = 0; j < la->n; j++)
                if (!la->e[j].worm && la->e[j].dir == d && la->e[j].tick > tcur) { t = la->e[j].tick; break; }
            if (t < 0) break;
            tcur = t;
            int k = slab_of(c, t);
            /* legs end at the temporal boundaries, so the slabs of a bond are
               independent updates.  Streams: unit (bond, slab); vertex v of
               the bond in the slab (tick order) draws its choice from kind
               RNG_BS and the worms of leg g from kind RNG_BSL + g, each from
               word 2^17 v on (word-pair index v << 16) */
            if (k != kcur) { kcur = k; v = 0; }
            const uint32_t unit = (uint32_t)(b * c->ntau + k);
            rstream s;
            rs_init(&s, c, RNG_BS, unit);
            s.w = (uint64_t)v << 17;
            int va = find_vertex(c, a, t, d), vc = find_vertex(c, cc, t, d + 2);
            if (va < 0 || vc < 0) { c->flags |= FLAG_STATE; return; }
            int32_t lo_a, lo_c, hi_a, hi_c;
            int p1, p2, q1, q2;
            leg_below(c, a, k, va, &lo_a, &p1);
            leg_below(c, cc, k, vc, &lo_c, &p2);
            leg_above(c, a, k, va, &hi_a, &q1);
            leg_above(c, cc, k, vc, &hi_c, &q2);
            int64_t l0 = (int64_t)t - lo_a, l1 = (int64_t)t - lo_c;
            int64_t l2 = (int64_t)hi_a - t, l3 = (int64_t)hi_c - t;
            double W[6];
            for (int m = 0; m < 6; m++) {
                int S = ALLOWED[m];
                int s1 = S & 1, s2 = (S >> 1) & 1, s1p = (S >> 2) & 1, s2p = S >> 3;
                W[m] = (((fleg(c, p1 ^ s1, l0) * fleg(c, p2 ^ s2, l1))
                         * fleg(c, s1p ^ q1, l2)) * fleg(c, s2p ^ q2, l3)) * vweight(c, S);
            }
            int m = choose(W, 6, u53(rs_next(&s)));
            int S = ALLOWED[m];
            int s1 = S & 1, s2 = (S >> 1) & 1, s1p = (S >> 2) & 1, s2p = S >> 3;
            /* new roots; then the worms on the four legs are regenerated */
            c->site[a].e[va].up = (uint8_t)s1p;
            c->site[cc].e[vc].up = (uint8_t)s2p;
            erase_worms(c, a, lo_a, t);
            erase_worms(c, cc, lo_c, t);
            erase_worms(c, a, t, hi_a);
            erase_worms(c, cc, t, hi_c);
            rstream sl[4];
            for (int g = 0; g < 4; g++) {
                rs_init(&sl[g], c, RNG_BSL + g, unit);
                sl[g].w = (uint64_t)v << 17;
            }
            place_worms(c, &sl[0], a, lo_a, l0, p1 ^ s1, p1);
            place_worms(c, &sl[1], cc, lo_c, l1, p2 ^ s2, p2);
            place_worms(c, &sl[2], a, t, l2, s1p ^ q1, s1p);
            place_worms(c, &sl[3], cc, t, l3, s2p ^ q2, s2p);
            v++;
        }
    }
}

/* ------------------------------------------------------------------ */
/* driver                                                              */
/* ------------------------------------------------------------------ */
static int validate(const orc_params* p)
{
    if (p->Lx < 3 || p->Ly < 3) return 0;
    if (!(p->beta > 0.0) || !(p->eta > 0.0) || !(p->t >= 0.0)) return 0;
    if (p->dom_x < 1 || p->dom_y < 1 || p->dom_tau < 1 || p->dom_tau > 64) return 0;
    if (p->Lx % p->dom_x || p->Ly % p->dom_y) return 0;
    if (p->Lx / p->dom_x < 2 || p->Ly / p->dom_y < 2) return 0;
    if (p->ticks_log2 < 8 || p->ticks_log2 > 30) return 0;
    if (((int64_t)1 << p->ticks_log2) / p->dom_tau < 2) return 0;
    if (p->chain_id >= (1u << 24)) return 0;
    if ((int64_t)p->Lx * p->Ly * p->dom_tau >= ((int64_t)1 << 30)) return 0;
    if (p->eta * p->beta > 50.0) return 0;
    return 1;
}

int orc_create(const orc_params* p, orc_chain** out)
{
    *out = NULL;
    if (!validate(p)) return ORC_EINVAL;
    orc_chain* c = (orc_chain*)calloc(1, sizeof(orc_chain));
    if (!c) return ORC_ENOMEM;
    c->p = *p;
    c->Lx = p->Lx; c->Ly = p->Ly; c->N = p->Lx * p->Ly;
    c->ntau = p->dom_tau;
    c->ex = p->Lx / p->dom_x; c->ey = p->Ly / p->dom_y;
    c->cdf = (double*)calloc((size_t)c->ntau * KMAX, sizeof(double));
    c->cdf_len = (int*)calloc((size_t)c->ntau, sizeof(int));
    c->site = (elist*)calloc((size_t)c->N, sizeof(elist));
    c->bstate = (uint8_t*)calloc((size_t)c->N * c->ntau, 1);
    c->bondv = (vlist*)calloc((size_t)2 * c->N, sizeof(vlist));
    if (!c->cdf || !c->cdf_len || !c->site || !c->bstate || !c->bondv) { orc_destroy(c); return ORC_ENOMEM; }
    build_tables(c);
    int ok = 1;
    for (int s = 0; s < 4; s++) if (!(c->wd[s] > 0.0)) ok = 0;
    if (!(c->rho_max * p->beta / c->ntau < 500.0)) ok = 0;
    if (c->ncycle < 1 || c->ncycle > 10000000) ok = 0;
    if (!ok) { orc_destroy(c); return ORC_EINVAL; }
    *out = c;
    return ORC_OK;
}

void orc_destroy(orc_chain* c)
{
    if (!c) return;
    if (c->site) for (int i = 0; i < c->N; i++) free(c->site[i].e);
    if (c->bondv) for (int64_t b = 0; b < 2 * (int64_t)c->N; b++) free(c->bondv[b].v);
    free(c->site); free(c->bondv); free(c->bstate); free(c->cdf); free(c->cdf_len);
    free(c->series);
    free(c);
}

static void record(orc_chain* c)
{
    if (c->nseries == c->capseries) {
        int64_t cap = c->capseries ? 2 * c->capseries : 1024;
        orc_obs* s = (orc_obs*)realloc(c->series, sizeof(orc_obs) * (size_t)cap);
        if (!s) { c->flags |= FLAG_NOMEM; return; }
        c->series = s; c->capseries = cap;
    }
    c->series[c->nseries++] = c->cur;
    /* running sums and sums of squares, in sweep order */
    orc_summary* a = &c->sums;
    const orc_obs* o = &c->cur;
    a->sweeps += 1;
    a->nv += o->nv; a->nkink += o->nkink; a->nw += o->nw; a->occ2 += o->occ2; a->nn2 += o->nn2;
    a->qimp = a->qimp + o->qimp;
    a->nv_sq = a->nv_sq + (double)o->nv * (double)o->nv;
    a->nkink_sq = a->nkink_sq + (double)o->nkink * (double)o->nkink;
    a->nw_sq = a->nw_sq + (double)o->nw * (double)o->nw;
    a->occ2_sq = a->occ2_sq + (double)o->occ2 * (double)o->occ2;
    a->nn2_sq = a->nn2_sq + (double)o->nn2 * (double)o->nn2;
    a->qimp_sq = a->qimp_sq + o->qimp * o->qimp;
    memset(&c->cur, 0, sizeof(c->cur));
}

void orc_reset_observables(orc_chain* c) { memset(&c->sums, 0, sizeof(c->sums)); }

static double sem(double sum, double sq, double S)
{
    if (!(S > 1.0)) return NAN;
    double m = sum / S;
    double var = sq / S - m * m;
    return sqrt((var > 0.0 ? var : 0.0) / (S - 1.0));
}

/* the estimators of the expansion of Tr exp(-beta H_eta) (C N_b - <number
   of operators>/beta for H_eta, <N_w>/beta for eta Q) and the improved
   worm-density estimator of Supplemental S-I */
int orc_observables(const orc_chain* c, orc_summary* out)
{
    *out = c->sums;
    double S = (double)c->sums.sweeps, N = (double)c->N, M = (double)c->M;
    double beta = c->p.beta, eta = c->p.eta, V = c->p.V, mu = c->p.mu;
    double m_nv = (double)c->sums.nv / S, m_nk = (double)c->sums.nkink / S;
    double m_nw = (double)c->sums.nw / S, m_occ = (double)c->sums.occ2 / S;
    double m_nn = (double)c->sums.nn2 / S, m_q = c->sums.qimp / S;
    out->E = 2.0 * c->C - m_nv / (beta * N);
    out->E_alt = (V * m_nn - mu * m_occ) / (2.0 * M * N) - m_nk / (beta * N);
    out->E_eta = out->E - m_nw / (beta * N);
    out->density = m_occ / (2.0 * M * N);
    out->Q = m_nw / (beta * eta * N);
    out->Q_imp = m_q / (M * N);
    out->b = 0.5 * out->Q_imp;
    out->err_E = sem((double)c->sums.nv, c->sums.nv_sq, S) / (beta * N);
    out->err_density = sem((double)c->sums.occ2, c->sums.occ2_sq, S) / (2.0 * M * N);
    out->err_Q = sem((double)c->sums.nw, c->sums.nw_sq, S) / (beta * eta * N);
    out->err_Q_imp = sem(c->sums.qimp, c->sums.qimp_sq, S) / (M * N);
    return c->flags ? ORC_ESTATE : ORC_OK;
}

int orc_phase(orc_chain* c, int phase)
{
    switch (phase) {
    case ORC_PH_V:   vertex_phase(c); break;
    case ORC_PH_R:   worm_phase_R(c); break;
    case ORC_PH_S:   scatter_phase(c); break;
    case ORC_PH_BT:  temporal_phase(c); break;
    case ORC_PH_BSX: spatial_phase(c, 0); break;
    case ORC_PH_BSY: spatial_phase(c, 1); break;
    case ORC_PH_END: record(c); c->sweep++; break;
    default: return ORC_EINVAL;
    }
    return c->flags ? ORC_ESTATE : ORC_OK;
}

int orc_sweep(orc_chain* c, int64_t n)
{
    for (int64_t s = 0; s < n; s++)
        for (int ph = ORC_PH_V; ph <= ORC_PH_END; ph++) {
            int r = orc_phase(c, ph);
            if (r) return r;
        }
    return ORC_OK;
}

int64_t orc_series(orc_chain* c, orc_obs* out, int64_t max_rows)
{
    int64_t n = c->nseries < max_rows ? c->nseries : max_rows;
    if (n > 0) memcpy(out, c->series, sizeof(orc_obs) * (size_t)n);
    memmove(c->series, c->series + n, sizeof(orc_obs) * (size_t)(c->nseries - n));
    c->nseries -= n;
    return n;
}

int orc_flags(const orc_chain* c) { return c->flags; }

/* ------------------------------------------------------------------ */
/* canonical state                                                     */
/* ------------------------------------------------------------------ */
int64_t orc_state_events(const orc_chain* c)
{
    int64_t n = 0;
    for (int i = 0; i < c->N; i++) n += c->site[i].n;
    return n;
}

int orc_get_state(const orc_chain* c, uint8_t* bstate, int32_t* counts,
                  int32_t* ticks, uint32_t* infos, int64_t cap, uint64_t* sweep)
{
    if (orc_state_events(c) > cap) return ORC_EINVAL;
    memcpy(bstate, c->bstate, (size_t)c->N * c->ntau);
    int64_t o = 0;
    for (int k = 0; k < c->ntau; k++)
        for (int i = 0; i < c->N; i++) {
            int lo, hi;
            slab_range(c, i, k, &lo, &hi);
            counts[(size_t)k * c->N + i] = hi - lo;
            for (int j = lo; j < hi; j++) {
                const ev_t* e = &c->site[i].e[j];
                ticks[o] = e->tick;
                infos[o] = (uint32_t)e->worm | ((uint32_t)e->dir << 1) | ((uint32_t)e->up << 3);
                o++;
            }
        }
    *sweep = c->sweep;
    return ORC_OK;
}

int orc_set_state(orc_chain* c, const uint8_t* bstate, const int32_t* counts,
                  const int32_t* ticks, const uint32_t* infos, int64_t n_events,
                  uint64_t sweep)
{
    memcpy(c->bstate, bstate, (size_t)c->N * c->ntau);
    for (int i = 0; i < c->N; i++) c->site[i].n = 0;
    int64_t o = 0;
    for (int k = 0; k < c->ntau; k++)
        for (int i = 0; i < c->N; i++) {
            int n = counts[(size_t)k * c->N + i];
            for (int j = 0; j < n; j++) {
                if (o >= n_events) return ORC_EINVAL;
                ev_t e = { ticks[o], (uint8_t)(infos[o] & 1),
                           (uint8_t)((infos[o] >> 1) & 3), (uint8_t)((infos[o] >> 3) & 1) };
                elist* l = &c->site[i];
                el_reserve(c, l, l->n + 1);
                if (c->flags & FLAG_NOMEM) return ORC_ENOMEM;
                l->e[l->n++] = e;
                o++;
            }
        }
    c->sweep = sweep;
    memset(&c->cur, 0, sizeof(c->cur));
    memset(&c->sums, 0, sizeof(c->sums));
    return ORC_OK;
}

/* worldline invariants: sorted keys, distinct worm slots, each slab
   propagates from its boundary state to the next one (flips exactly at
   worms and kinks), both ends of every vertex agree on flip / no flip,
   vertex roots form an allowed vertex state */
int orc_check(const orc_chain* c)
{
    int bad = 0;
    for (int i = 0; i < c->N; i++) {
        const elist* l = &c->site[i];
        for (int j = 0; j < l->n; j++) {
            const ev_t* e = &l->e[j];
            if (e->tick < 0 || e->tick >= c->M) bad++;
            if (j > 0) {
                int64_t bid = e->worm ? 0 : bond_id(c, i, e->dir);
                if (key_cmp(c, i, &l->e[j - 1], e->tick, e->worm, bid) >= 0) bad++;
            }
        }
        for (int k = 0; k < c->ntau; k++) {
            int lo, hi;
            slab_range(c, i, k, &lo, &hi);
            int st = c->bstate[(size_t)k * c->N + i];
            for (int j = lo; j < hi; j++) {
                const ev_t* e = &l->e[j];
                if (e->worm) { if (e->up == st) bad++; }
                else {
                    int a = e->dir < 2 ? i : nb(c, i, e->dir);
                    int bd = e->dir & 1;
                    int cc = nb(c, a, bd);
                    int va = find_vertex(c, a, e->tick, bd);
                    int vc = find_vertex(c, cc, e->tick, bd + 2);
                    if (va < 0 || vc < 0) { bad++; }
                    else {
                        int S = state_below(c, a, k, va) | (state_below(c, cc, k, vc) << 1)
                              | (c->site[a].e[va].up << 2) | (c->site[cc].e[vc].up << 3);
                        if (!(vweight(c, S) > 0.0)) bad++;
                    }
                }
                st = e->up;
            }
            if (st != c->bstate[(size_t)((k + 1) % c->ntau) * c->N + i]) bad++;
        }
    }
    return bad;
}

static uint64_t splitmix_final(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

uint64_t orc_state_hash(const orc_chain* c)
{
    uint64_t h = 0;
    for (int k = 0; k < c->ntau; k++)
        for (int i = 0; i < c->N; i++) {
            int lo, hi;
            slab_range(c, i, k, &lo, &hi);
            uint64_t u = (uint64_t)k * (uint64_t)c->N + (uint64_t)i;
            h += splitmix_final((u << 20) ^ ((uint64_t)(hi - lo) << 1) ^ (uint64_t)c->bstate[(size_t)k * c->N + i]);
            for (int j = lo; j < hi; j++) {
                const ev_t* e = &c->site[i].e[j];
                uint64_t info = (uint64_t)e->worm | ((uint64_t)e->dir << 1) | ((uint64_t)e->up << 3);
                h += splitmix_final(splitmix_final((u << 15) | (uint64_t)(j - lo))
                                    ^ (((uint64_t)(uint32_t)e->tick << 4) | info));
            }
        }
    return h;
}

int orc_get_derived(const orc_chain* c, orc_derived* d)
{
    d->C = c->C; d->rho_max = c->rho_max; d->lambda = c->lambda; d->delta = c->delta;
    for (int s = 0; s < 4; s++) { d->wd[s] = c->wd[s]; d->acc[s] = c->acc[s]; }
    d->n_cycle = c->ncycle; d->M = c->M; d->ntau = c->ntau;
    for (int k = 0; k <= c->ntau; k++) d->T[k] = c->T[k];
    return ORC_OK;
}

int orc_get_scatter_table(const orc_chain* c, double* tab, double* pair)
{
    memcpy(tab, c->scat, sizeof(c->scat));
    memcpy(pair, c->pairw, sizeof(c->pairw));
    return ORC_OK;
}

int orc_poisson_table(const orc_chain* c, int k, double* cdf, int cap)
{
    if (k < 0 || k >= c->ntau) return ORC_EINVAL;
    int n = c->cdf_len[k];
    for (int j = 0; j < n && j < cap; j++) cdf[j] = c->cdf[(size_t)k * KMAX + j];
    return n;
}

/* ------------------------------------------------------------------ */
/* worms of one interval for a general local operator                  */
/* (Eq. (worm) and the sequence rule after it, general form)           */
/* ------------------------------------------------------------------ */
#define GQ_TERMS 256
enum { RNG_GQ = 10 };

/* Draws the worms of an interval I of `ell` free half-tick slots whose end
   states are p (bottom) and q (top), for Q = sum_alpha Q_alpha given as
   nonnegative d x d matrices, x = I*eta = lam*ell:

   1. the count n with probability x^n/n! <q|Q^n|p> / f_qp, where
      f_qp = <q|exp(x Q)|p> is summed as a series of the scaled vectors
      u_j = (x^j/j!) Q^j |p>;
   2. n distinct uniform slots, sorted (as for hard-core worms);
   3. the sequence: worm k (time order) carries the type alpha_k and takes
      the state from s_{k-1} to s_k; the path (alpha_k, s_k) is drawn with
      probability prod_k <s_k|Q_{alpha_k}|s_{k-1}> / <q|Q^n|p>, from the last
      worm back to the first: given s_k, (alpha_k, s_{k-1}) is chosen with
      weight <s_k|Q_{alpha_k}|s_{k-1}> <s_{k-1}|Q^{k-1}|p>;
   4. one direction bit per worm in ascending slot order. */
int orc_worms_general(const orc_localq* g, double lam, int64_t ell, int p, int q,
                      uint64_t seed, uint32_t stream, uint32_t sweep, uint32_t unit,
                      int cap, int32_t* slots, uint8_t* alpha, uint8_t* after, uint8_t* dirs)
{
    int d = g->d, na = g->nalpha;
    if (d < 2 || d > ORC_GQ_DMAX || na < 1 || na > ORC_GQ_AMAX) return ORC_EINVAL;
    if (p < 0 || p >= d || q < 0 || q >= d || ell < 0 || cap < 0 || cap > ORC_GQ_CAPMAX)
        return ORC_EINVAL;
    if (!(lam >= 0.0) || !isfinite(lam) || stream >= (1u << 24)) return ORC_EINVAL;
    double Q[ORC_GQ_DMAX][ORC_GQ_DMAX];
    for (int a = 0; a < d; a++)
        for (int b = 0; b < d; b++) {
            double s = 0.0;
            for (int al = 0; al < na; al++) {
                double v = g->q[al][a][b];
                if (!(v >= 0.0) || !isfinite(v)) return ORC_EINVAL;
                s = s + v;
            }
            Q[a][b] = s;
        }
    if (ell == 0) return p == q ? 0 : ORC_ESTATE;

    /* y bounds the growth of the 1-norm: |Q v|_1 <= qn |v|_1 for v >= 0 */
    double qn = 0.0;
    for (int b = 0; b < d; b++) {
        double s = 0.0;
        for (int a = 0; a < d; a++) s = s + Q[a][b];
        if (s > qn) qn = s;
    }
    double x = lam * (double)ell;
    double y = x * qn;

    /* series of f_qp; stop after term j once j + 2 >= 2y and the remaining
       terms, at most 2 y |u_j|_1 / (j + 1), are below 2^-60 of the sum */
    double u[GQ_TERMS][ORC_GQ_DMAX];
    double tq[GQ_TERMS];
    for (int a = 0; a < d; a++) u[0][a] = (a == p) ? 1.0 : 0.0;
    double S = 0.0;
    int J = -1;
    for (int j = 0; j < GQ_TERMS; j++) {
        if (j > 0) {
            double c = x / (double)j;
            for (int a = 0; a < d; a++) {
                double s = 0.0;
                for (int b = 0; b < d; b++) s = s + Q[a][b] * u[j - 1][b];
                u[j][a] = c * s;
            }
        }
        tq[j] = u[j][q];
        S = S + tq[j];
        double norm = 0.0;
        for (int a = 0; a < d; a++) norm = norm + u[j][a];
        if ((double)(j + 2) >= 2.0 * y &&
            (norm == 0.0 || (S > 0.0 && 2.0 * y * norm / (double)(j + 1) <= 0x1p-60 * S))) {
            J = j;
            break;
        }
    }
    if (J < 0) return ORC_EINVAL;            /* x |Q| too large for the series */
    if (!(S > 0.0)) return ORC_ESTATE;       /* q cannot be reached from p     */
    double f = S;

    rstream s;
    s.key[0] = (uint32_t)seed; s.key[1] = (uint32_t)(seed >> 32);
    s.ctr[0] = 0; s.ctr[1] = unit; s.ctr[2] = sweep; s.ctr[3] = (stream << 8) | RNG_GQ;
    s.w = 0; s.have = 0; s.blk = 0;

    /* 1. the count */
    int n = -1;
    for (int tries = 0; tries < 1000 && n < 0; tries++) {
        double U = u53(rs_next(&s)) * f;
        double cum = 0.0;
        for (int j = 0; j <= J; j++) {
            cum = cum + tq[j];
            if (U < cum) {
                if ((int64_t)j <= ell) n = j;
                break;
            }
        }
    }
    if (n < 0) return ORC_ESTATE;
    if (n > cap) return ORC_ECAP;

    /* 2. the slots */
    for (int i = 0; i < n; i++) {
        int32_t r;
        int again, guard = 0;
        do {
            r = (int32_t)below(rs_next(&s), (uint64_t)ell);
            again = 0;
            for (int k = 0; k < i; k++) if (slots[k] == r) { again = 1; break; }
        } while (again && ++guard < 100000);
        if (again) return ORC_ESTATE;
        slots[i] = r;
    }
    for (int a = 1; a < n; a++) {
        int32_t v = slots[a]; int b = a - 1;
        while (b >= 0 && slots[b] > v) { slots[b + 1] = slots[b]; b--; }
        slots[b + 1] = v;
    }

    /* 3. the sequence, from the last worm back to the first */
    int st = q;
    for (int k = n; k >= 1; k--) {
        double T = 0.0;
        for (int al = 0; al < na; al++)
            for (int b = 0; b < d; b++) T = T + g->q[al][st][b] * u[k - 1][b];
        if (!(T > 0.0)) return ORC_ESTATE;
        double U = u53(rs_next(&s)) * T;
        double cum = 0.0;
        int ca = -1, cb = -1, la = -1, lb = -1;
        for (int al = 0; al < na && ca < 0; al++)
            for (int b = 0; b < d; b++) {
                double w = g->q[al][st][b] * u[k - 1][b];
                if (w > 0.0) { la = al; lb = b; }
                cum = cum + w;
                if (U < cum) { ca = al; cb = b; break; }
            }
        if (ca < 0) { ca = la; cb = lb; }   /* U rounded up to T */
        alpha[k - 1] = (uint8_t)ca;
        after[k - 1] = (uint8_t)st;
        st = cb;
    }
    if (st != p) return ORC_ESTATE;

    /* 4. the directions */
    for (int i = 0; i < n; i++) dirs[i] = (uint8_t)(rs_next(&s) >> 63);
    return n;
}
