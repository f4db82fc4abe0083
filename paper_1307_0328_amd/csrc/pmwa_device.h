// pmwa_device.h -- device-side data layout and helpers of the gfx950 PMWA
// sweep (Masaki-Kato et al., arXiv:1307.0328).
//
// Layout in device memory, per chain (all offsets are into shared pools):
//   site-slab unit  u = (k * ndsp + dsp) * nloc + sl      (k temporal slab,
//                   dsp spatial domain, sl site inside the domain, row-major)
//   events          ev[ev_off + ((k*ndsp + dsp) * cap + j) * nloc + sl]
//                   j-th event of the site in slab k, stored {tick, info};
//                   consecutive sites of a domain are consecutive in memory,
//                   so lane-per-site kernels read coalesced rows.
//   counts          cnt[cnt_off + u]
//   boundary state  bs[bs_off + u]       occupation just above T_k
//   bond buffer     bv[bv_off + (((k*2 + d)*ndsp + dsp) * capb + j) * nloc + sl]
//                   vertices of bond (site, +d) in slab k after the vertex
//                   phase, in tick order: tick | kink << 29 | s_a << 30 |
//                   s_c << 31 (occupations just below the vertex)
//   event info      bit0 worm; bit3 occupation just above; vertex bits1-2 =
//                   bond direction seen from this site (0 +x, 1 +y, 2 -x,
//                   3 -y); worm bit1 = moving up.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pmwa.h"

#define PMWA_DEV __device__ __forceinline__

namespace pmwa {

constexpr int NT_MAX = 64;      // temporal domains
constexpr int KMAXC = 256;      // Poisson table entries = max candidates per bond-slab
constexpr int NWL = 48;         // worms drawn on one interval
constexpr int RW_POOL = 64;     // worm-offset pool of the wavefront re-generation and the
                                // spatial update (above NWL: the first pending lane always fits)
static_assert(NWL <= RW_POOL, "the worm-offset pool must hold the worms of one interval, "
                              "or the pool rounds of k_assemble_w and k_bspatial make no progress");
// lanes per workgroup of the lane-per-unit kernels (vertex phase, temporal
// boundaries).  Full wavefronts: with fewer lanes the same work takes more
// memory and LDS instructions per CU, which measured slower than leaving
// SIMDs idle.
constexpr int VL = 64;
constexpr uint32_t NONE = 0xFFFFFFFFu;
constexpr uint32_t PX_NIL = 0xFFFFFFu;          // no partner end (24-bit link of an HBM node)
constexpr uint32_t BV_TICK = (1u << 29) - 1u;   // bond-buffer entry: tick bits
constexpr uint32_t BV_KINK = 1u << 29;          //   kink (occupations flip)

// stream kinds in Philox counter word 3 (low byte)
// (the spatial update draws a vertex's choice from RNG_BS and the worms of
// its leg g from RNG_BSL + g)
enum : uint32_t { RNG_V = 1, RNG_R = 2, RNG_S = 3, RNG_BT = 4, RNG_BS = 5, RNG_BSL = 6 };
// sticky per-chain error flags
enum : uint32_t { FL_OVERFLOW = 1, FL_SAMPLER = 2, FL_STATE = 4 };
// node flags of the scattering phase (bits 0-3 equal the event info bits)
enum : uint32_t { F_WORM = 1, F_DIRUP = 2, F_UP = 8, F_SBOT = 16, F_STOP = 32, F_CROSS = 64 };

struct ChainDev {
    int32_t Lx, Ly, N, ntau, ex, ey, nloc, dom_x, dom_y, ndsp;
    int32_t M, ncycle, cap, capb, cdf_stride, scr_nodes;
    uint32_t chain_id, key0, key1, n_dom;
    double lambda, t;
    int64_t ev_off, cnt_off, bs_off, bv_off, bvc_off, dom_off, ser_off, cdf_off;
    int64_t scr_off;   // node scratch of the HBM scattering path (nodes)
    int64_t oc_off;    // per-domain rows of site counts and offsets (HBM scattering form)
    int64_t target;    // sweeps after which the chain stops
    int32_t active;    // 0: idle slot, every kernel skips the chain
    int32_t pad1_;
    int32_t T[NT_MAX + 1];
    int32_t pad_;
    double F[1024];    // expm1(lambda * v * 2^(8g)) at [g*256 + v]
    double acc[4];     // w_d / rho_max, index s_a | s_c << 1
    double vw[16];     // vertex weight by root pattern
    double scat[256];  // cumulative exit table [S0][entry][exit]
};

struct DomPart {
    long long nv, nkink, nw, occ2;
    double qimp;
    long long windows;   // evaluation windows of the scattering phase (diagnostic)
};

struct Pools {
    const ChainDev* cd;
    uint2* ev;
    int32_t* cnt;
    uint8_t* bs;
    uint32_t* bv;
    int32_t* bvc;
    DomPart* dpart;
    pmwa_obs* ser;
    const double* cdf;
    unsigned long long* sweep;   // per chain
    unsigned int* flags;         // per chain
    unsigned long long* nnacc;   // per chain
    pmwa_obs_acc* acc;           // per chain: sums and squares of the records
    // scattering-phase node scratch in HBM: 16-byte nodes {tick, next,
    // previous, partner << 8 | flags}, the worm list, the owner stamps
    uint4* s_nd;
    uint32_t* s_wl;
    uint32_t* s_own;
    int32_t* s_oc;               // per domain 2 * nloc + 2 ints: site offsets, counts
    int32_t series_cap;
    int32_t lds_bytes;           // dynamic LDS of the scattering kernel's LDS form
};

// per vertex of a cross bond in the spatial boundary update (in LDS)
struct BsVert {
    int32_t t, lo_a, lo_c;
    int32_t l[4];            // leg lengths: lower a, lower c, upper a, upper c
    uint32_t fl;             // bit0 p1 fixed, bit1 p2 fixed, bit2 q1, bit3 q2,
                             // bit4 previous vertex on a is the bond's, bit5 on c,
                             // bit6 next vertex on a is the bond's, bit7 on c
    uint32_t m4;             // choice index for (p1, p2) = (x & 1, x >> 1) at bits 4x
    uint32_t S, p12;         // chosen root pattern; actual lower-end occupations
    uint8_t cnt[4];          // worms drawn on each leg, <= NWL (0 for legs redrawn later)
};
static_assert(NWL <= 255, "a leg's worm count is held in one byte");

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11)
// ---------------------------------------------------------------------------
PMWA_DEV void philox10(uint32_t x0, uint32_t x1, uint32_t x2, uint32_t x3,
                       uint32_t k0, uint32_t k1, uint32_t o[4])
{
#pragma unroll
    for (int r = 0; r < 10; r++) {
        // one 32x32 -> 64-bit product each (a single multiply-add instruction)
        const uint64_t p0 = (uint64_t)0xD2511F53u * x0, p1 = (uint64_t)0xCD9E8D57u * x2;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0, y2 = hi0 ^ x3 ^ k1;
        x0 = y0; x1 = lo1; x2 = y2; x3 = lo0;
        k0 += 0x9E3779B9u; k1 += 0xBB67AE85u;
    }
    o[0] = x0; o[1] = x1; o[2] = x2; o[3] = x3;
}

// N rounds of the same generator on a state carried between calls, the round
// keys advancing with it: ten rounds from (counter, key) equal philox10.
// Splitting the rounds lets a caller place them between dependent loads.
template <int N>
PMWA_DEV void philox_rounds(uint32_t (&x)[4], uint32_t& k0, uint32_t& k1)
{
#pragma unroll
    for (int r = 0; r < N; r++) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * x[0], p1 = (uint64_t)0xCD9E8D57u * x[2];
        const uint32_t y0 = (uint32_t)(p1 >> 32) ^ x[1] ^ k0, y2 = (uint32_t)(p0 >> 32) ^ x[3] ^ k1;
        x[1] = (uint32_t)p1; x[3] = (uint32_t)p0; x[0] = y0; x[2] = y2;
        k0 += 0x9E3779B9u; k1 += 0xBB67AE85u;
    }
}

// Word stream of one unit: word 2j = out1:out0, word 2j+1 = out3:out2 of the
// block with counter (j, unit, sweep, chain_id << 8 | kind).
struct Stream {
    uint32_t k0, k1, c1, c2, c3, w, blk;
    uint32_t o[4];
    PMWA_DEV void init(const ChainDev& C, uint32_t sweep, uint32_t kind, uint32_t unit)
    {
        k0 = C.key0; k1 = C.key1; c1 = unit; c2 = sweep; c3 = (C.chain_id << 8) | kind;
        w = 0; blk = 0;
    }
    // the same, from the chain's keys and id held by the caller
    PMWA_DEV void init_keys(uint32_t key0, uint32_t key1, uint32_t chain_id, uint32_t sweep, uint32_t kind,
                            uint32_t unit)
    {
        k0 = key0; k1 = key1; c1 = unit; c2 = sweep; c3 = (chain_id << 8) | kind;
        w = 0; blk = 0;
    }
    PMWA_DEV uint64_t next()
    {
        uint32_t j = w >> 1;
        if (blk != j + 1) { philox10(j, c1, c2, c3, k0, k1, o); blk = j + 1; }
        uint64_t r = (w & 1) ? (((uint64_t)o[3] << 32) | o[2]) : (((uint64_t)o[1] << 32) | o[0]);
        w++;
        return r;
    }
};

// The same word stream drawn by a whole wavefront in lock step: lane l
// computes block 64*b + l of batch b; words are read back with readlane.
struct WaveStream {
    uint32_t k0, k1, c1, c2, c3, w;
    uint32_t o0, o1, o2, o3;
    PMWA_DEV void init(const ChainDev& C, uint32_t sweep, uint32_t kind, uint32_t unit)
    {
        k0 = C.key0; k1 = C.key1; c1 = unit; c2 = sweep; c3 = (C.chain_id << 8) | kind;
        w = 0;
    }
    PMWA_DEV uint64_t next()
    {
        const uint32_t b = w & 127u;
        if (b == 0) {
            uint32_t o[4];
            philox10(((w >> 7) << 6) + (uint32_t)threadIdx.x, c1, c2, c3, k0, k1, o);
            o0 = o[0]; o1 = o[1]; o2 = o[2]; o3 = o[3];
        }
        const int ln = (int)(b >> 1);
        uint32_t lo, hi;
        if (b & 1u) { lo = __builtin_amdgcn_readlane(o2, ln); hi = __builtin_amdgcn_readlane(o3, ln); }
        else { lo = __builtin_amdgcn_readlane(o0, ln); hi = __builtin_amdgcn_readlane(o1, ln); }
        w++;
        return ((uint64_t)hi << 32) | lo;
    }
};

// SplitMix64 finaliser (the mixing function of the state hash)
PMWA_DEV uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

PMWA_DEV double u53(uint64_t w) { return (double)(w >> 11) * 0x1.0p-53; }
PMWA_DEV uint64_t below(uint64_t w, uint64_t n) { return __umul64hi(w, n); }

// ---------------------------------------------------------------------------
// lattice
// ---------------------------------------------------------------------------
PMWA_DEV int nbr(const ChainDev& C, int site, int d)
{
    int x = site % C.Lx, y = site / C.Lx;
    if (d == 0) x = (x + 1 == C.Lx) ? 0 : x + 1;
    else if (d == 1) y = (y + 1 == C.Ly) ? 0 : y + 1;
    else if (d == 2) x = (x == 0) ? C.Lx - 1 : x - 1;
    else y = (y == 0) ? C.Ly - 1 : y - 1;
    return y * C.Lx + x;
}
PMWA_DEV long long bond_id(const ChainDev& C, int site, int d)
{
    if (d < 2) return 2LL * site + d;
    return 2LL * nbr(C, site, d) + (d - 2);
}
PMWA_DEV void site_split(const ChainDev& C, int site, int& dsp, int& sl)
{
    int x = site % C.Lx, y = site / C.Lx;
    dsp = (y / C.ey) * C.dom_x + x / C.ex;
    sl = (y % C.ey) * C.ex + x % C.ex;
}
PMWA_DEV int site_join(const ChainDev& C, int dsp, int sl)
{
    int dy = dsp / C.dom_x, dx = dsp - dy * C.dom_x;
    int ly = sl / C.ex, lx = sl - ly * C.ex;
    return (dy * C.ey + ly) * C.Lx + dx * C.ex + lx;
}
PMWA_DEV long long unit_su(const ChainDev& C, int k, int dsp, int sl)
{
    return (long long)(k * C.ndsp + dsp) * C.nloc + sl;
}
PMWA_DEV long long ev_base(const ChainDev& C, int k, int dsp, int sl)
{
    return C.ev_off + (long long)(k * C.ndsp + dsp) * C.cap * C.nloc + sl;
}

// ---------------------------------------------------------------------------
// element functions of the worm law (hard-core f_qp), from the expm1 table
// ---------------------------------------------------------------------------
// F[g*256 + v] = expm1(lambda * v * 2^(8g)) (a copy in LDS); the base-256
// digits of ell in ascending order, (1+m)(1+t) - 1 = (m + t) + m t.  A zero
// digit has t = +0 and leaves m (finite, >= 0) unchanged exactly, so every
// digit is combined without a branch and the four loads issue together.
PMWA_DEV double em1(const double* __restrict__ F, long long ell)
{
    const double t0 = F[(int)(ell & 255)];
    const double t1 = F[256 + (int)((ell >> 8) & 255)];
    const double t2 = F[512 + (int)((ell >> 16) & 255)];
    const double t3 = F[768 + (int)((ell >> 24) & 255)];
    double m = t0;
    m = (m + t1) + m * t1;
    m = (m + t2) + m * t2;
    m = (m + t3) + m * t3;
    return m;
}
PMWA_DEV double fleg(const double* __restrict__ E, int sigma, long long ell)
{
    const double m = em1(E, ell);
    const double d = 2.0 * (1.0 + m);
    // the numerator selected first: one division whatever the mix of sigma
    // over a wavefront (sinh: m (2 + m) / d, cosh: 1 + m m / d)
    const double r = (sigma ? m * (2.0 + m) : m * m) / d;
    return sigma ? r : 1.0 + r;
}
PMWA_DEV double tanh_ell(const double* __restrict__ E, long long ell)
{
    double m = em1(E, ell);
    double d = 2.0 * (1.0 + m);
    return (m * (2.0 + m)) / (d + m * m);
}

// heat-bath choice: first m with W_m > 0 and u*sum < cumulative, else the
// last m with W_m > 0
template <int N>
PMWA_DEV int choose(const double (&W)[N], double u)
{
    double tot = 0.0;
    for (int m = 0; m < N; m++) tot = tot + W[m];
    double r = u * tot, cum = 0.0;
    int last = -1, pick = -1;
    for (int m = 0; m < N; m++) {
        cum = cum + W[m];
        if (W[m] > 0.0) {
            last = m;
            if (pick < 0 && r < cum) pick = m;
        }
    }
    return pick >= 0 ? pick : last;
}

// Sorts 32 values held in registers ascending (bitonic network; every index
// is a constant after unrolling, so nothing leaves the registers).
PMWA_DEV void sort32(int32_t (&c)[32])
{
#pragma unroll
    for (int k = 2; k <= 32; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
#pragma unroll
            for (int i = 0; i < 32; i++) {
                const int l = i ^ j;
                if (l > i) {
                    const int32_t a = c[i], b = c[l];
                    const int32_t lo = a < b ? a : b, hi = a < b ? b : a;
                    if ((i & k) == 0) { c[i] = lo; c[l] = hi; }
                    else { c[i] = hi; c[l] = lo; }
                }
            }
        }
    }
}

// Sorts v[0], v[ST], ..., v[ST(n-1)] (one lane's column of an LDS array)
// ascending; returns true when two entries are equal.
template <int ST = 64>
PMWA_DEV bool sort_col(int32_t* v, int n)
{
    bool rep = false;
    for (int x = 1; x < n; x++) {
        const int32_t t = v[x * ST];
        int y = x - 1;
        int32_t w = v[y * ST];
        while (w > t) {
            v[(y + 1) * ST] = w;
            if (--y < 0) break;
            w = v[y * ST];
        }
        rep |= (y >= 0 && w == t);
        v[(y + 1) * ST] = t;
    }
    return rep;
}

// Worms of one interval with `ell` free slots and end-state parity sigma:
// count by inversion of x^n/n!/f_sigma(x), x = lambda*ell, n <= ell (redraw
// otherwise); distinct uniform offsets in [0, ell), sorted; one direction
// bit per worm in ascending order.  The count and the slots are two calls on
// the same stream (the words follow each other as in one call).
// worm_count returns n, or -1 on failure (flagged).
template <class RS>
PMWA_DEV int worm_count(const double* __restrict__ E, double lambda, RS& s, long long ell, int sigma,
                        unsigned int* flag)
{
    if (ell == 0) {
        if (sigma) atomicOr(flag, FL_SAMPLER);
        return 0;
    }
    double f = fleg(E, sigma, ell);
    double x = lambda * (double)ell;
    double xx = x * x;
    long long nmax = ell < 4096 ? ell : 4096;
    int n = -1;
    for (int tries = 0; tries < 1000; tries++) {
        double U = u53(s.next()) * f;
        long long k = sigma;
        double T = sigma ? x : 1.0;
        double S = T;
        while (!(U < S) && k + 2 <= nmax) {
            T = (T * xx) / (double)((k + 1) * (k + 2));
            k += 2;
            S = S + T;
        }
        if (U < S && k <= nmax) { n = (int)k; break; }
    }
    if (n < 0 || n > NWL) { atomicOr(flag, FL_SAMPLER); return -1; }
    return n;
}

// a lane's column of offsets: entries i * ST of an LDS array
template <int ST>
struct LdsCol {
    int32_t* p;
    PMWA_DEV int32_t get(int i) const { return p[i * ST]; }
    PMWA_DEV void set(int i, int32_t v) const { p[i * ST] = v; }
};

// the n slots: offsets to col entries 0..n-1 (sorted), direction bit i to
// bit i of `dirs`.  Returns false on failure (flagged).
template <class RS, class Col>
PMWA_DEV bool worm_slots_col(RS& s, long long ell, int n, const Col& col, uint64_t& dirs, unsigned int* flag)
{
    dirs = 0;
    for (int i = 0; i < n; i++) {
        int32_t r;
        bool again;
        int guard = 0;
        do {
            r = (int32_t)below(s.next(), (uint64_t)ell);
            again = false;
            for (int j = 0; j < i; j++) again |= (col.get(j) == r);
        } while (again && ++guard < 100000);
        if (again) { atomicOr(flag, FL_SAMPLER); return false; }
        col.set(i, r);
    }
    for (int x = 1; x < n; x++) {            // insertion sort
        const int32_t t = col.get(x);
        int y = x - 1;
        while (y >= 0 && col.get(y) > t) {
            col.set(y + 1, col.get(y));
            y--;
        }
        col.set(y + 1, t);
    }
    for (int i = 0; i < n; i++) dirs |= (s.next() >> 63) << i;
    return true;
}

template <int ST, class RS>
PMWA_DEV bool worm_slots(RS& s, long long ell, int n, int32_t* off, uint64_t& dirs, unsigned int* flag)
{
    return worm_slots_col(s, ell, n, LdsCol<ST>{off}, dirs, flag);
}

// the same draws for n <= 2, the sorted offsets in registers
template <class RS>
PMWA_DEV bool worm_slots_reg(RS& s, long long ell, int n, int32_t& r0, int32_t& r1, uint64_t& dirs,
                             unsigned int* flag)
{
    dirs = 0;
    r0 = (int32_t)below(s.next(), (uint64_t)ell);
    if (n == 2) {
        int guard = 0;
        do {
            r1 = (int32_t)below(s.next(), (uint64_t)ell);
        } while (r1 == r0 && ++guard < 100000);
        if (r1 == r0) { atomicOr(flag, FL_SAMPLER); return false; }
        if (r1 < r0) { const int32_t t = r0; r0 = r1; r1 = t; }
    }
    for (int i = 0; i < n; i++) dirs |= (s.next() >> 63) << i;
    return true;
}

// the chain takes part in this sweep
PMWA_DEV bool live(const Pools& P, const ChainDev& C, int c)
{
    return C.active != 0 && P.flags[c] == 0 && P.sweep[c] < (unsigned long long)C.target;
}

// event encoding
PMWA_DEV uint32_t ev_worm(uint32_t info) { return info & 1u; }
PMWA_DEV uint32_t ev_dir(uint32_t info) { return (info >> 1) & 3u; }
PMWA_DEV uint32_t ev_up(uint32_t info) { return (info >> 3) & 1u; }
PMWA_DEV long long pos2(uint2 e) { return 2LL * (int)e.x + (long long)(e.y & 1u); }

}  // namespace pmwa
