// pmwa_kernels.hip -- gfx950 kernels of one PMWA sweep (Masaki-Kato et al.,
// arXiv:1307.0328): vertex phase (Step 3), worm re-generation (Step 4),
// worm scattering with measurement (Steps 5-6, Supplemental S-I), temporal
// (Step 1, Eq. (Para)) and spatial (Step 2, Eq. (ParaSpace)) boundary updates.
//
// Every kernel takes a block table {chain, first unit}: a block never spans
// two chains, so one launch advances any mix of lattices.
#include "pmwa_device.h"

namespace pmwa {

// ===========================================================================
// Step 3: vertex phase.  One lane per (bond, slab): keep the kinks, draw a
// Poisson(rho_max * Delta * dT_k) number of candidate ticks, and accept each
// with w_d(state)/rho_max (thinning gives the density of the diagonal matrix
// element).  Also integrates n_a n_c over the slab (before the update).  The
// bond's kinks and accepted vertices go to its bond buffer in tick order.
// ===========================================================================
PMWA_DEV bool key_before(const ChainDev& C, int site, uint2 e, int32_t tick, long long bid)
{
    int32_t et = (int32_t)e.x;
    if (et != tick) return et < tick;
    if (ev_worm(e.y)) return false;
    return bond_id(C, site, (int)ev_dir(e.y)) < bid;
}

// Object lists of the two ends of a bond, as seen by the vertex phase.  A
// record packs tick | worm << 29 | up << 30 | m << 31, with up the occupation
// just above the object and m = it is a vertex of the bond's direction d.
// Only objects that change the occupation (kinks and worms) matter for the
// states seen by candidates, for the n_a n_c integral and for the kinks kept,
// so FlipList holds just those (in LDS); FullList reads all events from HBM.
struct FlipList {
    const uint32_t* r;   // LDS column: tick | worm << 29 | dir << 30
    int n, s0, d;
    PMWA_DEV uint32_t get(int j) const
    {
        const uint32_t x = r[j * VL];
        const uint32_t w = (x >> 29) & 1u;
        const uint32_t up = (uint32_t)(s0 ^ ((j + 1) & 1));
        const uint32_t m = (!w && (int)(x >> 30) == d) ? 1u : 0u;
        return (x & (BV_TICK | (1u << 29))) | (up << 30) | (m << 31);
    }
    PMWA_DEV int dir(int j) const { return (int)(r[j * VL] >> 30); }
};
struct FullList {
    const uint2* E;
    int n, st, d;
    PMWA_DEV uint32_t get(int j) const
    {
        const uint2 e = E[(long long)j * st];
        const uint32_t w = e.y & 1u;
        const uint32_t m = (!w && (int)((e.y >> 1) & 3u) == d) ? 1u : 0u;
        return e.x | (w << 29) | (((e.y >> 3) & 1u) << 30) | (m << 31);
    }
    PMWA_DEV int dir(int j) const { return (int)ev_dir(E[(long long)j * st].y); }
};

PMWA_DEV long long pk_pos2(uint32_t pe) { return 2LL * (long long)(pe & BV_TICK) + (long long)((pe >> 29) & 1u); }
PMWA_DEV int pk_up(uint32_t pe) { return (int)((pe >> 30) & 1u); }

// the object ordered before the candidate (tau, bid) on `site`?  Equal ticks
// between vertices are decided by bond id.
template <class Lst>
PMWA_DEV bool pk_before(const ChainDev& C, int site, uint32_t pe, const Lst& L, int j, int32_t tau, long long bid)
{
    const int32_t t = (int32_t)(pe & BV_TICK);
    if (t != tau) return t < tau;
    if (pe & (1u << 29)) return false;
    return bond_id(C, site, L.dir(j)) < bid;
}

struct BondCtx {
    int a, c, sa0, sc0, st;
    long long bid;
};

// One ordered pass over the objects of both ends, with the sorted candidates
// cand[0..np) (a lane column of LDS: tick | rank << 29, the rank being the
// number of acceptance thresholds at or below the candidate's word) taken at
// their place in the site order.  Kinks of the bond and accepted candidates are written to `out` in
// tick order.  With INTEG, also integrates n_a n_c in half ticks over
// [2 T_k, 2 T_k+1).  A candidate on the tick of a kink of the bond stops the
// candidates (returns -1; the integral is still completed); otherwise
// returns the number of entries.
template <bool INTEG, class Lst>
PMWA_DEV int bond_walk(const ChainDev& C, const BondCtx& B, const Lst& LA, const Lst& LC,
                       int32_t Tk, int32_t Tk1, const int32_t* cand, int np, uint32_t acc_cnt,
                       uint32_t* out, int capb, long long& nn)
{
    int ia = 0, ic = 0, s_a = B.sa0, s_c = B.sc0, i = 0, nout = 0;
    bool clash = false;
    long long last = 2LL * Tk;
    uint32_t ea = LA.n > 0 ? LA.get(0) : 0u;
    uint32_t ec = LC.n > 0 ? LC.get(0) : 0u;
    const uint32_t cw0 = np > 0 ? (uint32_t)cand[0] : 0u;
    int32_t tau = (int32_t)(cw0 & BV_TICK);
    uint32_t rank = cw0 >> 29;
    for (;;) {
        const bool ha = ia < LA.n, hc = ic < LC.n;
        const bool pend = i < np;
        const bool ka = pend && ha && pk_before(C, B.a, ea, LA, ia, tau, B.bid);
        const bool kc = pend && hc && pk_before(C, B.c, ec, LC, ic, tau, B.bid);
        if (pend && !ka && !kc) {
            // every object ordered before the candidate has been passed
            if (ha && (int32_t)(ea & BV_TICK) == tau && (ea >> 31) && pk_up(ea) != s_a) {
                clash = true;
                np = i;
                if (!INTEG) break;
                continue;
            }
            // accepted iff its word is below the threshold of the state
            const int sidx = s_a | (s_c << 1);
            const uint32_t need = (acc_cnt >> (3 * sidx)) & 7u;
            if (rank < need) {
                if (nout < capb) out[(long long)nout * B.st] = (uint32_t)tau | ((uint32_t)s_a << 30) | ((uint32_t)s_c << 31);
                nout++;
            }
            i++;
            if (i < np) { const uint32_t cw = (uint32_t)cand[i * VL]; tau = (int32_t)(cw & BV_TICK); rank = cw >> 29; }
            continue;
        }
        if (!ha && !hc) break;
        if (!INTEG && !pend && !ha) break;   // only kinks of the bond are left to copy
        const bool takea = pend ? (ka && (!kc || pk_pos2(ea) <= pk_pos2(ec)))
                                : (!hc || (ha && pk_pos2(ea) <= pk_pos2(ec)));
        if (INTEG) {
            const long long p = pk_pos2(takea ? ea : ec);
            nn += (long long)(s_a & s_c) * (p - last);
            last = p;
        }
        if (takea) {
            const int up = pk_up(ea);
            if (!clash && (ea >> 31) && up != s_a) {
                if (nout < capb)
                    out[(long long)nout * B.st] = (ea & BV_TICK) | BV_KINK | ((uint32_t)s_a << 30) | ((uint32_t)(s_a ^ 1) << 31);
                nout++;
            }
            s_a = up;
            ia++;
            if (ia < LA.n) ea = LA.get(ia);
        } else {
            s_c = pk_up(ec);
            ic++;
            if (ic < LC.n) ec = LC.get(ic);
        }
    }
    if (INTEG) nn += (long long)(s_a & s_c) * (2LL * Tk1 - last);
    return clash ? -1 : nout;
}

// bit dir set: the bond of `site` in direction dir orders before bond `bid`
PMWA_DEV uint32_t bond_before_mask(const ChainDev& C, int site, long long bid)
{
    uint32_t m = 0;
#pragma unroll
    for (int dir = 0; dir < 4; dir++) m |= (bond_id(C, site, dir) < bid ? 1u : 0u) << dir;
    return m;
}

// bond_walk<true> on flip lists in LDS columns, as a merge on integer keys:
// key = 4 tick + class, the class being 1 for the candidate, 0 for a vertex
// whose bond orders before the candidate's bond, 2 for a vertex whose bond
// orders after it, 3 for a worm (worms sit on the half-tick slot above).  A
// flip precedes the candidate exactly when its key is smaller.  Flips of the
// two ends at one position may be taken in either order: the n_a n_c
// integral gains nothing between them and only flips of end a write output.
// Each step advances one of the three streams (one LDS read through a
// selected pointer).  Same result and the same -1 on a clash.
PMWA_DEV int bond_walk_flips(const BondCtx& B, const uint32_t* __restrict__ FA, int na,
                             const uint32_t* __restrict__ FC, int nc, uint32_t mask_a, uint32_t mask_c,
                             uint32_t d, int32_t Tk, int32_t Tk1, const int32_t* cand, int np, uint32_t acc_cnt,
                             uint32_t* out, int capb, long long& nn)
{
    const uint32_t INF = 0xFFFFFFFFu;
    // class of a flip record: 3 for a worm, else 0 or 2 by the mask bit of
    // its direction (a 2-bit table indexed by worm << 1 | mask bit)
    auto fkey = [](uint32_t r, uint32_t mask) -> uint32_t {
        const uint32_t w = (r >> 29) & 1u, m = (mask >> (r >> 30)) & 1u;
        return ((r & BV_TICK) << 2) | ((0xF2u >> ((w << 2) | (m << 1))) & 3u);
    };
    int ia = 0, ic = 0, i = 0, nout = 0, oidx = 0;
    uint32_t s_a = (uint32_t)B.sa0, s_c = (uint32_t)B.sc0;
    bool clash = false;
    int32_t last = 2 * Tk;                  // positions in half ticks (< 2^31)
    int32_t acc = 0;                        // the slab's integral, below 2^31
    const uint32_t kink_tag = d << 1;       // bits 29.. of a vertex of this bond
    uint32_t ra = na > 0 ? FA[0] : 0u, rc = nc > 0 ? FC[0] : 0u;
    uint32_t rx = np > 0 ? (uint32_t)cand[0] : 0u;
    uint32_t ka = na > 0 ? fkey(ra, mask_a) : INF;
    uint32_t kc = nc > 0 ? fkey(rc, mask_c) : INF;
    uint32_t kx = np > 0 ? (((rx & BV_TICK) << 2) | 1u) : INF;
    while ((ka & kc & kx) != INF) {
        // which stream comes next (keys of different streams differ, but
        // for equal flip keys, where end a goes first); every update below
        // is a select, so the lanes of a wavefront stay together
        const uint32_t km = min(min(ka, kc), kx);
        const bool isx = kx == km;
        const bool isa = !isx & (ka == km);
        const bool isc = !isx & !isa;
        const uint32_t tau = rx & BV_TICK, rank = rx >> 29;
        const bool a_kink = (ra >> 29) == kink_tag;   // a vertex of this bond
        // a candidate on the tick of the next kink of this bond on end a
        const bool cl = isx & a_kink & (ka == ((tau << 2) | 2u));
        const uint32_t need = (acc_cnt >> (3u * (s_a | (s_c << 1)))) & 7u;
        // (bitwise operators throughout: no short-circuit branches)
        const bool wr = (isx & !cl & (rank < need)) | (isa & !clash & a_kink);
        const uint32_t val = isx ? (tau | (s_a << 30) | (s_c << 31))
                                 : ((ra & BV_TICK) | BV_KINK | (s_a << 30) | ((s_a ^ 1u) << 31));
        if (wr & (nout < capb)) out[oidx] = val;
        nout += wr ? 1 : 0;
        oidx += wr ? B.st : 0;
        // n_a n_c integral up to a flip
        const uint32_t rf = isa ? ra : rc;
        const int32_t pos = 2 * (int32_t)(rf & BV_TICK) + (int32_t)((rf >> 29) & 1u);
        acc += (!isx & ((s_a & s_c) != 0u)) ? pos - last : 0;
        last = isx ? last : pos;
        s_a ^= isa ? 1u : 0u;
        s_c ^= isc ? 1u : 0u;
        clash |= cl;
        i += (isx & !cl) ? 1 : 0;
        ia += isa ? 1 : 0;
        ic += isc ? 1 : 0;
        // next record of the stream that advanced: one LDS read, from row 0
        // past the end of the list (every column has a row 0)
        const int nx = isx ? i : isa ? ia : ic;
        const int lim = isx ? np : isa ? na : nc;
        const uint32_t* src = isx ? reinterpret_cast<const uint32_t*>(cand) : isa ? FA : FC;
        const uint32_t rn = src[(nx < lim ? nx : 0) * VL];
        const uint32_t kn = nx < lim ? (isx ? (((rn & BV_TICK) << 2) | 1u) : fkey(rn, isa ? mask_a : mask_c)) : INF;
        rx = isx ? rn : rx;
        kx = isx ? (cl ? INF : kn) : kx;
        ra = isa ? rn : ra;
        ka = isa ? kn : ka;
        rc = isc ? rn : rc;
        kc = isc ? kn : kc;
    }
    acc += (s_a & s_c) ? 2 * Tk1 - last : 0;
    nn += acc;
    return clash ? -1 : nout;
}

// Acceptance with probability w_d(state)/rho_max by the word w: u53(w) <
// acc[s] is the same as (w >> 11) < ceil(acc[s] * 2^53) (exact integers), so
// a word is summarised by its rank r = number of the four thresholds at or
// below w >> 11, and the candidate is accepted in state s iff r < cnt[s],
// cnt[s] = number of thresholds at or below the threshold of s.
struct AccRank {
    uint64_t thr[4];
    uint32_t cnt;        // cnt[s] in bits 3s..3s+2
    PMWA_DEV void init(const ChainDev& C)
    {
#pragma unroll
        for (int q = 0; q < 4; q++) thr[q] = (uint64_t)ceil(C.acc[q] * 0x1.0p53);
        cnt = 0;
#pragma unroll
        for (int q = 0; q < 4; q++) {
            uint32_t c = 0;
#pragma unroll
            for (int r = 0; r < 4; r++) c += thr[r] <= thr[q] ? 1u : 0u;
            cnt |= c << (3 * q);
        }
    }
    PMWA_DEV uint32_t rank(uint64_t w) const
    {
        const uint64_t m = w >> 11;
        return (thr[0] <= m ? 1u : 0u) + (thr[1] <= m ? 1u : 0u) + (thr[2] <= m ? 1u : 0u) + (thr[3] <= m ? 1u : 0u);
    }
};

// the acceptance words of the sorted candidates follow the tick words
PMWA_DEV void tag_ranks(int32_t* cand, int n, Stream& rs, const AccRank& AR)
{
    for (int i = 0; i < n; i++) cand[i * VL] = (int32_t)((uint32_t)cand[i * VL] | (AR.rank(rs.next()) << 29));
}

// kinks of the bond, exact sequential candidate draws (a tick on a kink of
// the bond or on an earlier candidate is drawn again), then the pass
template <class Lst>
PMWA_DEV int vertex_exact(const ChainDev& C, const BondCtx& B, const Lst& LA, const Lst& LC,
                          int32_t Tk, int32_t Tk1, int32_t* cand, int n, uint32_t sweep, uint32_t unit,
                          const AccRank& AR, uint32_t* out, int capb, unsigned int* flag)
{
    // the kinks are listed in the bond buffer first (it is rewritten below)
    int nk = 0;
    {
        int s = B.sa0;
        for (int j = 0; j < LA.n; j++) {
            const uint32_t pe = LA.get(j);
            const int up = pk_up(pe);
            if ((pe >> 31) && up != s) {
                if (nk < capb) out[(long long)nk * B.st] = pe & BV_TICK;
                nk++;
            }
            s = up;
        }
    }
    if (nk > capb) { atomicOr(flag, FL_OVERFLOW); nk = capb; }
    Stream rs;
    rs.init(C, sweep, RNG_V, unit);
    (void)rs.next();
    const uint64_t dT = (uint64_t)(Tk1 - Tk);
    for (int i = 0; i < n; i++) {
        int32_t tau;
        bool again;
        int guard = 0;
        do {
            tau = Tk + (int32_t)below(rs.next(), dT);
            again = false;
            for (int j = 0; j < nk; j++) again |= ((int32_t)out[(long long)j * B.st] == tau);
            for (int j = 0; j < i; j++) again |= (cand[j * VL] == tau);
        } while (again && ++guard < 100000);
        if (again) { atomicOr(flag, FL_SAMPLER); n = i; break; }
        cand[i * VL] = tau;
    }
    sort_col<VL>(cand, n);
    tag_ranks(cand, n, rs, AR);
    long long unused = 0;
    const int nout = bond_walk<false>(C, B, LA, LC, Tk, Tk1, cand, n, AR.cnt, out, capb, unused);
    if (nout < 0) { atomicOr(flag, FL_STATE); return 0; }
    return nout;
}

// occupation-changing objects (kinks and worms) of both ends of a bond ->
// their LDS columns (at most `rows` each).  Branch-free body: every event is
// written at the next free row and kept only if it changes the occupation.
// Each batch issues the loads of up to 16 events of each end together, from
// positions clamped to the list (a list with no events reads its first slot,
// which is allocated), so that one round trip to memory serves the batch;
// only the events inside the lists count.  Returns the two counts (which may
// exceed rows).
PMWA_DEV int2 stage_flips(const uint2* EA, int na, int sa0, uint32_t* FA,
                           const uint2* EC, int nc, int sc0, uint32_t* FC, int st, int rows)
{
    constexpr int SB = 16;
    int fa = 0, fc = 0, s_a = sa0, s_c = sc0;
    const int nmax = na > nc ? na : nc;
    const int la = na > 0 ? na - 1 : 0, lc = nc > 0 ? nc - 1 : 0;
    for (int j = 0; j < nmax; j += SB) {
        uint2 ea[SB], ec[SB];
#pragma unroll
        for (int q = 0; q < SB; q++) {
            ea[q] = EA[(long long)(j + q < la ? j + q : la) * st];
            ec[q] = EC[(long long)(j + q < lc ? j + q : lc) * st];
        }
#pragma unroll
        for (int q = 0; q < SB; q++) {
            const bool va = j + q < na, vc = j + q < nc;
            const int ua = (int)ev_up(ea[q].y), uc = (int)ev_up(ec[q].y);
            FA[(fa < rows ? fa : rows - 1) * VL] = ea[q].x | ((ea[q].y & 1u) << 29) | (((ea[q].y >> 1) & 3u) << 30);
            FC[(fc < rows ? fc : rows - 1) * VL] = ec[q].x | ((ec[q].y & 1u) << 29) | (((ec[q].y >> 1) & 3u) << 30);
            fa += (va && ua != s_a) ? 1 : 0;
            fc += (vc && uc != s_c) ? 1 : 0;
            s_a = va ? ua : s_a;
            s_c = vc ? uc : s_c;
        }
    }
    return make_int2(fa, fc);
}

// dynamic LDS: the Poisson tables of the first two slabs of the block (2 * vs
// doubles), then per lane a column of cr candidate rows followed by two
// columns of `rows` rows for the occupation-changing objects of both ends of
// the lane's bond.
// A lane with more than cr candidates (cr + 2 rows >= the table length)
// continues its candidate column into its flip columns and walks its site
// lists in HBM.
__global__ void __launch_bounds__(VL) k_vertex(Pools P, const int2* __restrict__ blk, int vs, int cr, int rows,
                                               int vmode)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int2 bt = blk[blockIdx.x];
    const ChainDev& C = P.cd[bt.x];
    const int lane = (int)threadIdx.x;
    const int u = bt.y + lane;
    double* s_cdf = reinterpret_cast<double*>(smem);
    int32_t* cand = reinterpret_cast<int32_t*>(smem + 2 * (size_t)vs * sizeof(double)) + lane;
    uint32_t* FA = reinterpret_cast<uint32_t*>(smem + 2 * (size_t)vs * sizeof(double)) + (size_t)cr * VL + lane;
    uint32_t* FC = FA + (size_t)rows * VL;
    const int k_first = bt.y / (2 * C.N);
#pragma unroll 4
    for (int i = lane; i < 2 * C.cdf_stride; i += VL) {
        const int kk = k_first + i / C.cdf_stride;
        s_cdf[i] = kk < C.ntau ? P.cdf[C.cdf_off + (long long)kk * C.cdf_stride + i % C.cdf_stride] : 2.0;
    }
    __syncthreads();
    long long nn = 0;
    if (u < 2 * C.ntau * C.N && live(P, C, bt.x)) {
        unsigned int* flag = &P.flags[bt.x];
        const int sl = u % C.nloc;
        int r = u / C.nloc;
        const int dsp = r % C.ndsp;
        r /= C.ndsp;
        const int d = r & 1, k = r >> 1;
        BondCtx B;
        B.a = site_join(C, dsp, sl);
        B.c = nbr(C, B.a, d);
        int dspc, slc;
        site_split(C, B.c, dspc, slc);
        B.bid = 2LL * B.a + d;
        B.st = C.nloc;
        const int na = P.cnt[C.cnt_off + unit_su(C, k, dsp, sl)];
        const int nc = P.cnt[C.cnt_off + unit_su(C, k, dspc, slc)];
        B.sa0 = P.bs[C.bs_off + unit_su(C, k, dsp, sl)];
        B.sc0 = P.bs[C.bs_off + unit_su(C, k, dspc, slc)];
        const uint2* Ea = P.ev + ev_base(C, k, dsp, sl);
        const uint2* Ec = P.ev + ev_base(C, k, dspc, slc);
        const int2 nf2 = stage_flips(Ea, na, B.sa0, FA, Ec, nc, B.sc0, FC, B.st, rows);
        const int nfa = nf2.x, nfc = nf2.y;
        // a column is used only with a row to spare: once a count reaches
        // `rows`, later events land on the last row, which then no longer
        // holds the last flip
        bool staged = nfa < rows && nfc < rows && !(vmode & 1);
        const FlipList fla{FA, nfa, B.sa0, d}, flc{FC, nfc, B.sc0, -1};
        const FullList gla{Ea, na, B.st, d}, glc{Ec, nc, B.st, -1};

        const int32_t Tk = C.T[k], Tk1 = C.T[k + 1];
        const uint32_t sweep = (uint32_t)P.sweep[bt.x];
        const uint32_t unit = (uint32_t)(B.bid * C.ntau + k);
        const int capb = C.capb;
        uint32_t* out = P.bv + C.bv_off + (long long)((k * 2 + d) * C.ndsp + dsp) * capb * C.nloc + sl;

        Stream rs;
        rs.init(C, sweep, RNG_V, unit);
        const double u0 = u53(rs.next());
        // candidate count: the first n with u0 < cdf[n].  The table does not
        // decrease and ends in 2.0 entries, so a binary search finds it in a
        // fixed number of steps
        int n;
        {
            const double* cdf = k - k_first < 2 ? s_cdf + (k - k_first) * C.cdf_stride
                                                : P.cdf + C.cdf_off + (long long)k * C.cdf_stride;
            int lo = 0, hi = C.cdf_stride - 1;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (u0 < cdf[mid]) hi = mid;
                else lo = mid + 1;
            }
            n = lo;
        }
        // more candidates than the column's rows: they run on into the flip
        // columns, and the walk reads the site lists from HBM
        if (n > cr) staged = false;
        const uint64_t dT = (uint64_t)(Tk1 - Tk);
        // ticks as first drawn; they are the ticks kept unless one repeats
        // a kink of the bond or another candidate.  Up to 32 candidates are
        // drawn, sorted (bitonic network) and ranked in registers; the stream
        // is read in the same order either way (the n tick words, then the
        // acceptance words of the sorted candidates)
        AccRank AR;
        AR.init(C);
        bool rep;
        if (n <= 32 && !(vmode & 2)) {
            // the draws stay rolled loops through the LDS column (unrolled,
            // each inlined generator call would multiply the code size)
            for (int i = 0; i < n; i++) cand[i * VL] = Tk + (int32_t)below(rs.next(), dT);
            int32_t c[32];
#pragma unroll
            for (int i = 0; i < 32; i++) c[i] = i < n ? cand[i * VL] : 0x7FFFFFFF;
            sort32(c);
            rep = false;
#pragma unroll
            for (int i = 0; i + 1 < 32; i++) rep |= (i + 1 < n) && c[i] == c[i + 1];
#pragma unroll
            for (int i = 0; i < 32; i++)
                if (i < n) cand[i * VL] = c[i];
            if (!rep) tag_ranks(cand, n, rs, AR);
        } else {
            for (int i = 0; i < n; i++) cand[i * VL] = Tk + (int32_t)below(rs.next(), dT);
            rep = sort_col<VL>(cand, n);
            if (!rep) tag_ranks(cand, n, rs, AR);
        }
        int nout;
        if (staged) {
            const uint32_t mask_a = bond_before_mask(C, B.a, B.bid), mask_c = bond_before_mask(C, B.c, B.bid);
            nout = bond_walk_flips(B, FA, nfa, FC, nfc, mask_a, mask_c, (uint32_t)d, Tk, Tk1, cand, rep ? 0 : n,
                                   AR.cnt, out, capb, nn);
        } else {
            nout = bond_walk<true>(C, B, gla, glc, Tk, Tk1, cand, rep ? 0 : n, AR.cnt, out, capb, nn);
        }
        if (rep || nout < 0)
            nout = staged ? vertex_exact(C, B, fla, flc, Tk, Tk1, cand, n, sweep, unit, AR, out, capb, flag)
                          : vertex_exact(C, B, gla, glc, Tk, Tk1, cand, n, sweep, unit, AR, out, capb, flag);
        if (nout > capb) { atomicOr(flag, FL_OVERFLOW); nout = capb; }
        P.bvc[C.bvc_off + (long long)((k * 2 + d) * C.ndsp + dsp) * C.nloc + sl] = nout;
    }
    // wave sum of the bond occupation integral -> one atomic per block
    for (int o = VL / 2; o > 0; o >>= 1) nn += __shfl_down(nn, o, 64);
    if (threadIdx.x == 0 && nn) atomicAdd(&P.nnacc[bt.x], (unsigned long long)nn);
}

// ===========================================================================
// Step 4: per (site, slab) merge the vertex lists of the four bonds of the
// site (kinks and new diagonal vertices, from the bond buffers) in (tick,
// bond id) order, and generate the worms of every interval with Eq. (worm);
// interval r (from the bottom) draws from word 2^17 r of the (site, slab)
// stream.  The site's old list (old vertices and worms) is overwritten.
// k_assemble: one lane per (site, slab); k_assemble_w: one wavefront.
// ===========================================================================
// a column of worm offsets kept in the .x words of a site's event slots
// (stride st), where the worms will be written
struct EvCol {
    uint2* p;
    long long st;
    PMWA_DEV int32_t get(int i) const { return (int32_t)p[i * st].x; }
    PMWA_DEV void set(int i, int32_t v) const { p[i * st].x = (uint32_t)v; }
};

__global__ void __launch_bounds__(64) k_assemble(Pools P, const int2* __restrict__ blk)
{
    const int2 bt = blk[blockIdx.x];
    const ChainDev& C = P.cd[bt.x];
    const int u = bt.y + (int)threadIdx.x;
    // the expm1 table is read from L2, and the kernel holds no LDS: more lane
    // groups share a CU
    const double* sE = C.F;
    if (u >= C.ntau * C.N || !live(P, C, bt.x)) return;
    unsigned int* flag = &P.flags[bt.x];
    const double lambda = C.lambda;
    const int sl = u % C.nloc;
    const int r = u / C.nloc;
    const int dsp = r % C.ndsp, k = r / C.ndsp;
    const int i = site_join(C, dsp, sl);
    const int st = C.nloc;
    uint2* E = P.ev + ev_base(C, k, dsp, sl);
    const long long cu = C.cnt_off + unit_su(C, k, dsp, sl);
    const int s_lo = P.bs[C.bs_off + unit_su(C, k, dsp, sl)];
    const int s_hi = P.bs[C.bs_off + unit_su(C, (k + 1) % C.ntau, dsp, sl)];

    // the four bond buffers of this site: (i,+x), (i,+y), (i-x,+x), (i-y,+y)
    const uint32_t* src[4];
    int ns[4], ps[4];
    long long bids[4];
    uint32_t hv[4];
#pragma unroll
    for (int d = 0; d < 4; d++) {
        const int a = (d < 2) ? i : nbr(C, i, d);
        int dspa, sla;
        site_split(C, a, dspa, sla);
        const int bd = d & 1;
        const long long row = (long long)((k * 2 + bd) * C.ndsp + dspa);
        src[d] = P.bv + C.bv_off + row * C.capb * C.nloc + sla;
        ns[d] = P.bvc[C.bvc_off + row * C.nloc + sla];
        ps[d] = 0;
        bids[d] = 2LL * a + bd;
        hv[d] = ns[d] > 0 ? src[d][0] : 0u;
    }
    Stream rs;
    rs.init(C, (uint32_t)P.sweep[bt.x], RNG_R, (uint32_t)((long long)i * C.ntau + k));
    int32_t lo = C.T[k];
    // read before the loop's event stores, which could alias fields of C
    const int32_t Tk1 = C.T[k + 1];
    const int capu = C.cap;
    int p = s_lo;
    int out = 0;
    uint32_t ri = 0;                // interval index: vertices passed so far
    for (;;) {
        // next vertex in (tick, bond id) order
        int best = -1;
        int32_t btk = 0;
        long long bb = 0;
#pragma unroll
        for (int d = 0; d < 4; d++) {
            const int32_t tk = (int32_t)(hv[d] & BV_TICK);
            if (ps[d] < ns[d] && (best < 0 || tk < btk || (tk == btk && bids[d] < bb))) {
                best = d; btk = tk; bb = bids[d];
            }
        }
        uint32_t v = 0;
#pragma unroll
        for (int d = 0; d < 4; d++) {
            if (d == best) {
                v = hv[d];
                ps[d]++;
                if (ps[d] < ns[d]) hv[d] = src[d][(long long)ps[d] * st];
            }
        }
        int32_t hi;
        int q, above = 0;
        if (best < 0) { hi = Tk1; q = s_hi; }
        else {
            hi = btk;
            q = (int)((best < 2 ? v >> 30 : v >> 31) & 1u);
            above = q ^ (int)((v >> 29) & 1u);
        }
        uint64_t dirs = 0;
        rs.w = ri << 17;            // interval ri draws from word 2^17 ri on
        rs.blk = 0;
        // the count, then the slots: one or two in registers; more (rare) are
        // drawn and sorted in place in the event slots they will occupy
        const long long ell = (long long)hi - lo;
        const int n = worm_count(sE, lambda, rs, ell, p ^ q, flag);
        if (n < 0) return;
        if (out + n + (best >= 0 ? 1 : 0) > capu) { atomicOr(flag, FL_OVERFLOW); return; }
        int32_t r0 = 0, r1 = 0;
        if (n > 2) {
            if (!worm_slots_col(rs, ell, n, EvCol{E + (long long)out * st, st}, dirs, flag)) return;
        } else if (n > 0) {
            if (!worm_slots_reg(rs, ell, n, r0, r1, dirs, flag)) return;
        }
        ri++;
        int s = p;
        for (int w = 0; w < n; w++) {
            s ^= 1;
            const int32_t o = n > 2 ? (int32_t)E[(long long)out * st].x : (w == 0 ? r0 : r1);
            E[(long long)out * st] = make_uint2((uint32_t)(lo + o),
                                                1u | ((uint32_t)((dirs >> w) & 1u) << 1) | ((uint32_t)s << 3));
            out++;
        }
        if (best < 0) break;
        E[(long long)out * st] = make_uint2((uint32_t)hi, ((uint32_t)best << 1) | ((uint32_t)above << 3));
        out++;
        lo = hi;
        p = above;
    }
    P.cnt[cu] = out;
}

// ===========================================================================
// Steps 5-6: worm scattering, N_cycle cycles over the domain's worm list,
// then the measurement.  One wavefront per space-time domain; the domain's
// worldlines become doubly linked node lists (per site, between two boundary
// sentinels) held in LDS with 16-bit links when they fit, else in an HBM
// scratch region with 32-bit links.
// ===========================================================================
// A node as the window evaluation reads it: tick and flags; and with its
// links (next, previous, partner end)
struct NodeRec {
    int32_t t;
    uint32_t f;
};
struct NodeAll {
    int32_t t;
    uint32_t f, nx, pv, px;
};

// Node store in device memory (the HBM form): 16-byte nodes {tick, next,
// previous, partner << 8 | flags}, so that every dependent level of the
// window evaluation reads one 128-bit word per node; one owner stamp per
// node (a separate array: also the setup's and the measurement's scratch).
struct HbmStore {
    uint4* nd;
    uint32_t* wl;    // worm list
    uint32_t* own;   // per-node scratch in HBM (rank tables, estimator intervals; stamps when sh = 0)
    uint32_t* stp;   // owner stamps: own (one per node, sh = 0), or in the block's LDS, one per
    int sh;          // node pair (sh = 1; sharing can only end a window early, as in LDS)
    static constexpr bool in_lds = false;
    PMWA_DEV NodeAll all(uint32_t i) const
    {
        const uint4 v = nd[i];
        NodeAll r;
        r.t = (int32_t)v.x;
        r.nx = v.y;
        r.pv = v.z;
        r.px = v.w >> 8;
        r.f = v.w & 255u;
        return r;
    }
    PMWA_DEV void put(uint32_t i, int32_t t, uint32_t f, uint32_t px)
    {
        nd[i].x = (uint32_t)t;
        nd[i].w = (px << 8) | f;
    }
    // new flags of a node whose tick is unchanged
    PMWA_DEV void put_fl(uint32_t i, int32_t, uint32_t f, uint32_t px) { nd[i].w = (px << 8) | f; }
    PMWA_DEV void set_nx(uint32_t i, uint32_t v) { nd[i].y = v; }
    PMWA_DEV void set_pv(uint32_t i, uint32_t v) { nd[i].z = v; }
    PMWA_DEV uint32_t* stamp(uint32_t i) { return stp + (i >> sh); }
    PMWA_DEV int stamps(int nn) const { return (nn + sh) >> sh; }
    PMWA_DEV uint32_t* stamp_base() { return stp; }
};

// Node store in LDS (the LDS form), 12 bytes a node: one 32-bit word
// (tick - T_k) << 5 | flags, 16-bit links (next, previous, partner end) and
// an owner stamp shared by the nodes 2m and 2m + 1 (sharing can only end a
// window early, never let a conflict through).  Flag bits 0-3 are those of
// the event info; bit 4 (F_SBOT) marks every node a worm bounces off: the
// sentinels at the slab ends and the vertices of crossing bonds.
struct LdsStore {
    uint32_t* w;
    uint16_t* nxt;
    uint16_t* prv;
    uint16_t* aux;
    uint16_t* wl;
    uint32_t* own;
    int32_t base;    // T_k
    static constexpr bool in_lds = true;
    PMWA_DEV NodeRec rec(uint32_t i) const
    {
        const uint32_t x = w[i];
        NodeRec r;
        r.t = base + (int32_t)(x >> 5);
        r.f = x & 31u;
        return r;
    }
    // (the fields a caller does not use are never loaded)
    PMWA_DEV NodeAll all(uint32_t i) const
    {
        const NodeRec r = rec(i);
        NodeAll a;
        a.t = r.t;
        a.f = r.f;
        a.nx = nxt[i];
        a.pv = prv[i];
        a.px = aux[i];
        return a;
    }
    PMWA_DEV void put(uint32_t i, int32_t t, uint32_t f, uint32_t) { w[i] = ((uint32_t)(t - base) << 5) | f; }
    PMWA_DEV void put_fl(uint32_t i, int32_t t, uint32_t f, uint32_t px) { put(i, t, f, px); }
    PMWA_DEV void set_nx(uint32_t i, uint32_t v) { nxt[i] = (uint16_t)v; }
    PMWA_DEV void set_pv(uint32_t i, uint32_t v) { prv[i] = (uint16_t)v; }
    PMWA_DEV uint32_t* stamp(uint32_t i) { return own + (i >> 1); }
    PMWA_DEV int stamps(int nn) const { return (nn + 1) >> 1; }
    PMWA_DEV uint32_t* stamp_base() { return own; }
};

// floor(w * n / 2^64) for n < 2^32, exact
PMWA_DEV uint32_t below32(uint64_t w, uint32_t n)
{
    const uint64_t lo = (uint64_t)(uint32_t)w * n;
    const uint64_t hi = (uint64_t)(uint32_t)(w >> 32) * n + (lo >> 32);
    return (uint32_t)(hi >> 32);
}

// The workgroup of the scattering kernel is one wavefront, and a wavefront's
// LDS instructions execute in issue order, so with the node store in LDS
// (16-bit links) a lane reads what another lane wrote or stamped by an
// earlier instruction without waiting for it; only the compiler must keep
// the program order of the accesses.  With the node store in HBM the full
// barrier (and its wait for the memory operations) stays.
template <class Store>
PMWA_DEV void wave_order()
{
    if constexpr (Store::in_lds) {
        asm volatile("" ::: "memory");
        __builtin_amdgcn_wave_barrier();
    } else {
        __syncthreads();
    }
}

// Steps 5-6 over windows of up to 64 consecutive attempts of the serial
// sequence (cycle-major, worm-list order).  Lane k evaluates attempt s0+k,
// its whole decision included, on the state at the start of the window.  A
// worm with fewer than 64 worms in its domain can appear several times in a
// window: a repeat is evaluated as if its earlier attempts in the window
// turned the worm round (a turn changes nothing but the worm's direction,
// which no other attempt reads); had one of them moved the worm, the move
// wrote the worm's old neighbours, which the repeat reads, so the repeat
// conflicts.  The first attempt whose read set meets a node an earlier move
// of the window writes ends the window (owner stamps, LDS atomicMax).
// Attempt s draws stream words 3s, 3s+1, 3s+2 (enter test, exit leg, landing
// slot), used or not.  The surviving moves touch disjoint nodes and are
// applied together, a worm's turns by its last surviving attempt; decisions
// and the final state equal those of the attempts made one at a time in
// order.
//
// One attempt (Step 5): a worm facing another worm, a temporal boundary or a
// boundary vertex reverses; facing an interior vertex it enters with
// probability L_min/L_i (legs measured without the moving worm, so L_min is
// the same before and after, Eq. (DB)), leaves by leg j with probability
// w_ji/w_i, lands on a uniform free slot of leg j and faces away from the
// vertex.
template <class Store>
PMWA_DEV long long scatter_windows(Store& A, uint64_t* __restrict__ ring, int NN, int nw, const ChainDev& C,
                                   uint32_t sweep, uint32_t D, const uint64_t* __restrict__ sthr,
                                   unsigned int* flag)
{
    long long windows = 0;
    const int lane = (int)threadIdx.x;
    const long long total = (long long)C.ncycle * nw;
    if (total > 0x50000000LL) { if (lane == 0) atomicOr(flag, FL_OVERFLOW); return 0; }
    // lane k holds attempt s0 + k: worm-list position iw0 + (k mod nw), with
    // k / nw earlier attempts of the same worm in the window
    const int lm = nw > 0 ? lane % nw : 0;
    const int rep = nw > 0 ? lane / nw : 0;
    const int m64 = nw > 0 ? 64 % nw : 0;
    const uint32_t k0 = C.key0, k1 = C.key1, c1 = D, c2 = sweep, c3 = (C.chain_id << 8) | RNG_S;
    uint32_t cur = 0, filled = 0, wid = 0;
    int iw0 = 0;                       // worm-list position of attempt s0
    for (long long s0 = 0; s0 < total;) {
        // words [cur, cur + 192) of the stream sit in the 512-word ring (a
        // catch-up after long windows; the window below normally keeps it full)
        while (filled < cur + 192u) {
            uint32_t o[4];
            philox10((filled >> 1) + (uint32_t)lane, c1, c2, c3, k0, k1, o);
            ring[(filled + 2u * lane) & 511u] = ((uint64_t)o[1] << 32) | o[0];
            ring[(filled + 2u * lane + 1u) & 511u] = ((uint64_t)o[3] << 32) | o[2];
            filled += 128u;
        }
        if (++wid == (1u << 23)) {
            for (int i = lane; i < A.stamps(NN); i += 64) A.stamp_base()[i] = 0u;
            wid = 1;
        }
        wave_order<Store>();
        const bool act = s0 + lane < total;
        // the attempt's three stream words, read with the first loads of the
        // window (the empty asm below consumes them before the decision, so
        // that they are not deferred behind the evaluation)
        const uint32_t myc = cur + 3u * (uint32_t)lane;
        const uint64_t wd0 = ring[myc & 511u], wd1 = ring[(myc + 1u) & 511u], wd2 = ring[(myc + 2u) & 511u];
        // ---- evaluate on the window's starting state.  Every lane evaluates,
        //      so that the reads form one straight chain; an inactive lane
        //      still names a worm of the list, and a blocked attempt reads
        //      nothing past x (its x- and y-side nodes fall back to the worm),
        //      so every index is a node of the domain.
        int iw = iw0 + lm;
        if (iw >= nw) iw -= nw;
        const uint32_t w = A.wl[iw];
        // the next 128 stream words, computed two rounds at a time while the
        // window's dependent reads are in flight (each pair is tied to the
        // values of one level of reads) and stored at the end if the ring has
        // room for them
        uint32_t po[4] = {(filled >> 1) + (uint32_t)lane, c1, c2, c3};
        uint32_t pk0 = k0, pk1 = k1;
        philox_rounds<2>(po, pk0, pk1);
        asm("" : "+v"(po[0]), "+v"(po[1]), "+v"(po[2]), "+v"(po[3]) : "v"(w));
        const NodeAll aw = A.all(w);
        const uint32_t fw = aw.f ^ ((rep & 1) ? F_DIRUP : 0u);
        const uint32_t pw = aw.pv;
        const uint32_t nn_ = aw.nx;
        philox_rounds<2>(po, pk0, pk1);
        asm("" : "+v"(po[0]), "+v"(po[1]), "+v"(po[2]), "+v"(po[3]) : "v"(fw), "v"(pw), "v"(nn_));
        const bool up = (fw & F_DIRUP) != 0;
        const uint32_t x = up ? nn_ : pw;
        const uint32_t wf = up ? pw : nn_;
        const NodeAll ax = A.all(x);
        const uint32_t fx = ax.f;
        const int32_t t = ax.t;
        const uint32_t ya = ax.px;
        const uint32_t xfa = up ? ax.nx : ax.pv;
        const NodeAll awf = A.all(wf);
        const int32_t t_wf = awf.t;
        const uint32_t f_wf = awf.f;
        philox_rounds<2>(po, pk0, pk1);
        asm("" : "+v"(po[0]), "+v"(po[1]), "+v"(po[2]), "+v"(po[3]) : "v"(fx), "v"(ya), "v"(xfa));
        const bool blocked = (fx & (F_WORM | F_SBOT | F_STOP | F_CROSS)) != 0;
        const uint32_t y = blocked ? w : ya;
        const uint32_t xf = blocked ? w : xfa;
        const NodeAll ay = A.all(y);
        const uint32_t fy = ay.f;
        const uint32_t yp = ay.pv;
        const uint32_t yn = ay.nx;
        const NodeAll axf = A.all(xf);
        const int32_t t_xf = axf.t;
        const uint32_t f_xf = axf.f;
        const NodeAll ayp = A.all(yp);
        const int32_t t_yp = ayp.t;
        const uint32_t f_yp = ayp.f;
        const int32_t t_yn = A.all(yn).t;
        philox_rounds<2>(po, pk0, pk1);
        asm("" : "+v"(po[0]), "+v"(po[1]), "+v"(po[2]), "+v"(po[3]) : "v"(fy), "v"(yp), "v"(yn));
        philox_rounds<2>(po, pk0, pk1);
        const bool xa = ((fx >> 1) & 3u) < 2u;
        int32_t Lxb, Lxa;
        if (up) { Lxb = t - (t_wf + (int32_t)(f_wf & F_WORM)); Lxa = t_xf - t; }
        else { Lxa = t_wf - t; Lxb = t - (t_xf + (int32_t)(f_xf & F_WORM)); }
        const int32_t Lyb = t - (t_yp + (int32_t)(f_yp & F_WORM));
        const int32_t Lya = t_yn - t;
        const int32_t L0 = xa ? Lxb : Lyb, L1 = xa ? Lyb : Lxb, L2 = xa ? Lxa : Lya, L3 = xa ? Lya : Lxa;
        int32_t Lmin = L0 < L1 ? L0 : L1;
        Lmin = L2 < Lmin ? L2 : Lmin;
        Lmin = L3 < Lmin ? L3 : Lmin;
        const int32_t Li = up ? Lxb : Lxa;
        const int i = up ? (xa ? 0 : 1) : (xa ? 2 : 3);
        // ---- the decision on the window's starting state: enter test, exit
        //      leg and landing slot (stream words 3s, 3s+1, 3s+2); computed
        //      by every lane, kept where the attempt is active and not blocked
        asm volatile("" ::"v"(wd0), "v"(wd1), "v"(wd2));
        // (and the speculative words here, so that they are not sunk to the
        // store at the end, where nothing would hide their latency)
        asm volatile("" ::"v"(po[0]), "v"(po[1]), "v"(po[2]), "v"(po[3]));
        const uint32_t r = below32(wd0, (uint32_t)Li);
        const bool moved = act && !blocked && (int32_t)r < Lmin;
        // vertex roots with the worm in place
        const uint32_t rxb = up ? (fw >> 3) & 1u : (f_xf >> 3) & 1u;
        const uint32_t rxa = (fx >> 3) & 1u;
        const uint32_t ryb = (f_yp >> 3) & 1u, rya = (fy >> 3) & 1u;
        const int S = xa ? (int)(rxb | (ryb << 1) | (rxa << 2) | (rya << 3))
                         : (int)(ryb | (rxb << 1) | (rya << 2) | (rxa << 3));
        const int S0 = S ^ (1 << i);
        // u53(word) < P  <=>  (word >> 11) < ceil(P 2^53), exactly; the
        // cumulative thresholds do not decrease, so the exit leg (the first j
        // with word < row[j]) is the number at or below the word
        const uint64_t w53 = wd1 >> 11;
        const uint64_t* row = sthr + S0 * 16 + i * 4;
        const uint64_t th0 = row[0], th1 = row[1], th2 = row[2];
        const int j = (int)(w53 >= th0) + (int)(w53 >= th1) + (int)(w53 >= th2);
        const int32_t Lj = (j & 2) ? ((j & 1) ? L3 : L2) : ((j & 1) ? L1 : L0);
        const uint32_t r2 = below32(wd2, (uint32_t)Lj);
        // leave leg i: above the end on x, that segment takes the worm's state
        const uint32_t fx_now = up ? fx : ((fx & ~F_UP) | (fw & F_UP));
        const bool on_x = ((j & 1) != 0) != xa;
        const bool above = j >= 2;
        const uint32_t Pn = above ? (on_x ? x : y) : (on_x ? (up ? wf : xf) : yp);
        const uint32_t Nn = above ? (on_x ? (up ? xf : wf) : yn) : (on_x ? x : y);
        const uint32_t fv = on_x ? fx_now : fy;
        const uint32_t fp = on_x ? (up ? f_wf : f_xf) : f_yp;
        const uint32_t newup = above ? (fv & F_UP) : ((fp & F_UP) ^ F_UP);
        const int32_t ntick = above ? t + (int32_t)r2 : t - 1 - (int32_t)r2;
        // ---- nodes a move writes: the worm's old and new neighbours (the
        //      vertex end it leaves is one of the old ones).  Anything reading
        //      the worm node itself reads one of its old neighbours.  A turn
        //      only flips its own worm's direction, which no other attempt of
        //      the window reads.  The first attempt that reads a node an
        //      earlier one writes ends the window.
        const uint32_t stamp = (wid << 8) | (uint32_t)(255 - lane);
        if (moved) {
            atomicMax(A.stamp(pw), stamp);
            atomicMax(A.stamp(nn_), stamp);
            atomicMax(A.stamp(Pn), stamp);
            atomicMax(A.stamp(Nn), stamp);
        }
        wave_order<Store>();
        // stamps of earlier windows are below wid << 8; in this window a
        // stamp exceeds the lane's own value exactly when an earlier lane set
        // it.  A blocked attempt's x- and y-side nodes are the worm and its
        // neighbours, so it tests the three nodes it reads.
        const uint32_t v = max(max(max(*A.stamp(w), *A.stamp(pw)), max(*A.stamp(nn_), *A.stamp(xf))),
                               max(max(*A.stamp(y), *A.stamp(yp)), *A.stamp(yn)));
        const bool conflict = !act || v > stamp;
        const unsigned long long cmask = __ballot(conflict);
        const int kc = cmask ? __ffsll((long long)cmask) - 1 : 64;
        // ---- apply the surviving attempts (disjoint nodes)
        if (lane < kc) {
            if (!moved) {
                if (lane + nw >= kc) A.put_fl(w, aw.t, fw ^ F_DIRUP, aw.px);   // the worm's last attempt here
            } else {
                // (x and y are the two ends of one vertex: both at tick t,
                // each the other's partner)
                if (!up) A.put_fl(x, t, fx_now, ya);
                A.set_nx(pw, nn_);
                A.set_pv(nn_, pw);
                if (above) A.put_fl(Pn, t, fv ^ F_UP, on_x ? ya : ay.px);
                A.put(w, ntick, F_WORM | (above ? F_DIRUP : 0u) | newup, aw.px);
                A.set_pv(w, Pn);
                A.set_nx(w, Nn);
                A.set_nx(Pn, w);
                A.set_pv(Nn, w);
            }
        }
        // the speculative words go in when the ring has room: this window
        // read [cur, cur + 192), and the block [filled, filled + 128) must not
        // wrap onto words not yet consumed
        if (filled <= cur + 384u) {
            ring[(filled + 2u * lane) & 511u] = ((uint64_t)po[1] << 32) | po[0];
            ring[(filled + 2u * lane + 1u) & 511u] = ((uint64_t)po[3] << 32) | po[2];
            filled += 128u;
        }
        wave_order<Store>();
        cur += 3u * (uint32_t)kc;
        s0 += kc;
        // (iw0 + kc) mod nw: lane kc's position offset, read from its register
        iw0 += kc < 64 ? __builtin_amdgcn_readlane(lm, kc & 63) : m64;
        if (iw0 >= nw) iw0 -= nw;
        windows++;
    }
    return windows;
}

// one-wavefront exclusive scan
PMWA_DEV int wave_excl_scan(int v, int& total)
{
    const int lane = (int)threadIdx.x;
    int x = v;
    for (int o = 1; o < 64; o <<= 1) {
        int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    total = __shfl(x, 63, 64);
    return x - v;
}

PMWA_DEV void scatter_domain(const Pools& P, const ChainDev& C, int chain, int D,
                             HbmStore A, uint64_t* __restrict__ ring,
                             int* __restrict__ off, int* __restrict__ cnt,
                             const uint64_t* __restrict__ sthr, const double* __restrict__ sE, int NE,
                             bool restore_oc)
{
    const int lane = (int)threadIdx.x;
    const int k = D / C.ndsp, dsp = D - k * C.ndsp;
    const int nloc = C.nloc, ex = C.ex, ey = C.ey;
    const uint32_t BOT = (uint32_t)NE, TOP = (uint32_t)(NE + nloc);
    const uint32_t NIL = 0xFFFFFFFFu;
    uint32_t* own = A.own;

    // Steps 1-3 take one lane per site and walk the site's events in order.
    // The vertices of a bond carry the same ticks on its two sites, so the
    // partner of the r-th vertex of direction d on site s is the r-th vertex
    // of direction d ^ 2 on the neighbouring site.  Before the windows start,
    // the owner-stamp array serves as scratch for those ranks: per site
    // (4 x 16 bit) the first rank slot of directions 1, 2, 3 and the vertex
    // count, then per site (from off[s]) the node of every vertex, grouped by
    // direction.
    uint16_t* vtab = reinterpret_cast<uint16_t*>(own);
    uint32_t* vnode = reinterpret_cast<uint32_t*>(vtab + 4 * nloc);

    // 1. nodes from the events (loads of consecutive sites are adjacent in
    //    HBM), the sentinels, and the vertex count per direction; vertices
    //    of bonds that leave the domain are marked as boundary vertices (a
    //    worm bounces off them)
    const int32_t Tk = C.T[k], Tk1 = C.T[k + 1];
    for (int s = lane; s < nloc; s += 64) {
        const int o = off[s], n = cnt[s];
        const int lx = s % ex, ly = s / ex;
        // bit vd set: the bond in direction vd leaves the domain
        const uint32_t crm = ((C.dom_x > 1 && lx == ex - 1) ? 1u : 0u) | ((C.dom_y > 1 && ly == ey - 1) ? 2u : 0u) |
                             ((C.dom_x > 1 && lx == 0) ? 4u : 0u) | ((C.dom_y > 1 && ly == 0) ? 8u : 0u);
        const uint2* E = P.ev + ev_base(C, k, dsp, s);
        int c0 = 0, c1 = 0, c2 = 0, c3 = 0;
        for (int j0 = 0; j0 < n; j0 += 16) {
            uint2 e[16];
#pragma unroll
            for (int u = 0; u < 16; u++)
                if (j0 + u < n) e[u] = E[(long long)(j0 + u) * nloc];
#pragma unroll
            for (int u = 0; u < 16; u++) {
                const int j = j0 + u;
                if (j < n) {
                    const uint32_t idx = (uint32_t)(o + j);
                    const uint32_t f = e[u].y & 15u;
                    const uint32_t vd = (f >> 1) & 3u;
                    const bool v = (f & F_WORM) == 0u;
                    const uint32_t fl = f | ((v && ((crm >> vd) & 1u)) ? F_CROSS : 0u);
                    A.nd[idx] = make_uint4(e[u].x, j + 1 < n ? idx + 1u : TOP + (uint32_t)s,
                                           j > 0 ? idx - 1u : BOT + (uint32_t)s, (PX_NIL << 8) | fl);
                    c0 += v && vd == 0u;
                    c1 += v && vd == 1u;
                    c2 += v && vd == 2u;
                    c3 += v && vd == 3u;
                }
            }
        }
        vtab[4 * s + 0] = (uint16_t)c0;
        vtab[4 * s + 1] = (uint16_t)(c0 + c1);
        vtab[4 * s + 2] = (uint16_t)(c0 + c1 + c2);
        vtab[4 * s + 3] = (uint16_t)(c0 + c1 + c2 + c3);
        const int bsv = P.bs[C.bs_off + unit_su(C, k, dsp, s)];
        A.nd[BOT + s] = make_uint4((uint32_t)Tk, n ? (uint32_t)o : TOP + s, NIL,
                                   (PX_NIL << 8) | F_SBOT | (bsv ? F_UP : 0u));
        A.nd[TOP + s] = make_uint4((uint32_t)Tk1, NIL, n ? (uint32_t)(o + n - 1) : BOT + s, (PX_NIL << 8) | F_STOP);
    }
    __syncthreads();
    // 2. vertex nodes by (site, direction, rank), and the worm list in
    //    (site, slot) order = node order; the flags are read in batches and
    //    every entry is written with predication
    int nw = 0;
    for (int base = 0; base < nloc; base += 64) {
        const int s = base + lane;
        const int nws = s < nloc ? cnt[s] - (int)vtab[4 * s + 3] : 0;
        int tot;
        const int wpos = nw + wave_excl_scan(nws, tot);
        if (s < nloc) {
            const int o = off[s], n = cnt[s];
            int r0 = 0, r1 = (int)vtab[4 * s], r2 = (int)vtab[4 * s + 1], r3 = (int)vtab[4 * s + 2];
            int rw = wpos;
            for (int j0 = 0; j0 < n; j0 += 8) {
                uint32_t fb[8];
#pragma unroll
                for (int u = 0; u < 8; u++) fb[u] = j0 + u < n ? A.nd[o + j0 + u].w & 255u : 0u;
#pragma unroll
                for (int u = 0; u < 8; u++) {
                    if (j0 + u < n) {
                        const uint32_t idx = (uint32_t)(o + j0 + u);
                        const uint32_t f = fb[u];
                        const uint32_t vd = (f >> 1) & 3u;
                        if (f & F_WORM) {
                            A.wl[rw++] = idx;
                        } else {
                            const int r = vd == 0u ? r0 : vd == 1u ? r1 : vd == 2u ? r2 : r3;
                            vnode[o + r] = idx;
                            r0 += vd == 0u;
                            r1 += vd == 1u;
                            r2 += vd == 2u;
                            r3 += vd == 3u;
                        }
                    }
                }
            }
        }
        nw += tot;
    }
    __syncthreads();
    // 3. partner ends of vertices: per site and inner direction, the r-th
    //    vertex of direction d is matched with the r-th vertex of direction
    //    d ^ 2 on the neighbour (independent iterations)
    bool bad3 = false;
    for (int s = lane; s < nloc; s += 64) {
        const int o = off[s];
        const int lx = s % ex, ly = s / ex;
        const int st[5] = {0, (int)vtab[4 * s], (int)vtab[4 * s + 1], (int)vtab[4 * s + 2], (int)vtab[4 * s + 3]};
#pragma unroll
        for (int d = 0; d < 4; d++) {
            const bool cross = d == 0 ? (C.dom_x > 1 && lx == ex - 1) : d == 1 ? (C.dom_y > 1 && ly == ey - 1)
                             : d == 2 ? (C.dom_x > 1 && lx == 0) : (C.dom_y > 1 && ly == 0);
            if (cross) continue;
            const int nb = d == 0 ? (lx == ex - 1 ? s - (ex - 1) : s + 1)
                         : d == 1 ? (ly == ey - 1 ? s - (ey - 1) * ex : s + ex)
                         : d == 2 ? (lx == 0 ? s + (ex - 1) : s - 1)
                                  : (ly == 0 ? s + (ey - 1) * ex : s - ex);
            const int pd = d ^ 2;
            const int nb_lo = pd == 0 ? 0 : (int)vtab[4 * nb + pd - 1];
            const int nb_hi = (int)vtab[4 * nb + pd];
            const int nown = st[d + 1] - st[d];
            bad3 |= nown != nb_hi - nb_lo;
            const int m_n = nown < nb_hi - nb_lo ? nown : nb_hi - nb_lo;
            const uint32_t* own_v = vnode + o + st[d];
            const uint32_t* nb_v = vnode + off[nb] + nb_lo;
#pragma unroll 4
            for (int r = 0; r < m_n; r++) {
                const uint32_t idx = (uint32_t)own_v[r];
                const uint32_t m = (uint32_t)nb_v[r];
                const uint4 vi = A.nd[idx];
                bad3 |= vi.x != A.nd[m].x;
                A.nd[idx].w = (m << 8) | (vi.w & 255u);
            }
        }
    }
    if (bad3) atomicOr(&P.flags[chain], FL_STATE);
    __syncthreads();
    if (__any(P.flags[chain] != 0)) return;

    // 4. N_cycle cycles, worms in list order, evaluated in windows
    for (int i = lane; i < A.stamps(NE + 2 * nloc); i += 64) A.stamp_base()[i] = 0u;
    __syncthreads();
    const long long windows = scatter_windows(A, ring, NE + 2 * nloc, nw, C, (uint32_t)P.sweep[chain],
                                              (uint32_t)D, sthr, &P.flags[chain]);
    if (restore_oc) {
        // the stamps took the LDS of the per-site counts and offsets: the
        // counts are read again (unchanged until the write-back below) and
        // scanned again
        __syncthreads();
        for (int s = lane; s < nloc; s += 64) cnt[s] = P.cnt[C.cnt_off + unit_su(C, k, dsp, s)];
        __syncthreads();
        int carry = 0;
        for (int base = 0; base < nloc; base += 64) {
            const int s = base + lane;
            const int v = s < nloc ? cnt[s] : 0;
            int tot;
            const int ex_ = wave_excl_scan(v, tot);
            if (s < nloc) off[s] = carry + ex_;
            carry += tot;
        }
        if (lane == 0) off[nloc] = carry;
        __syncthreads();
    }

    // 5. measurement (Step 6) and write-back.  One lane per site follows the
    //    site's node list and writes the events back; the length and worm
    //    parity of every interval between vertices go to a table (the owner
    //    stamps' memory; vertices never leave their site, so site s has at
    //    most cnt[s] + 1 intervals, from slot off[s] + s), whose terms of the
    //    improved worm-density estimator all lanes then evaluate at once.
    uint32_t* qint = own;
    const int NN = NE + 2 * nloc;
    for (int i = lane; i < NN; i += 64) qint[i] = 0u;
    __syncthreads();
    // chain fields in registers: the loop's global stores could otherwise
    // alias them and force reloads
    const int capc = C.cap;
    const long long cnt_base = C.cnt_off + unit_su(C, k, dsp, 0);
    const long long ev_base0 = ev_base(C, k, dsp, 0);
    long long nv = 0, nkink = 0, nwc = 0, occ = 0;
    bool bad = false;
    for (int s = lane; s < nloc; s += 64) {
        const long long ebase = ev_base0 + s;
        uint32_t* qi = qint + off[s] + s;
        const int qmax = cnt[s] + 1;
        int nq = 0;
        int stt = (int)((A.nd[BOT + s].w >> 3) & 1u);
        int32_t lastp = 2 * Tk;                 // positions in half ticks (< 2^31)
        int32_t ilo = Tk;
        uint32_t par = 0;
        int j = 0;
        uint32_t node = A.nd[BOT + s].y;
        int guard = 0;
        // this site's tallies (the occupation integral is below 2^31)
        int occs = 0, nvs = 0, nks = 0, nws = 0;
        for (;;) {
            if (node == TOP + (uint32_t)s) {
                occs += stt * (2 * Tk1 - lastp);
                if (nq < qmax) qi[nq] = ((uint32_t)(Tk1 - ilo) << 1) | par;
                else bad = true;
                break;
            }
            if (node >= (uint32_t)NE || ++guard > NE) { bad = true; break; }
            const uint4 vn = A.nd[node];
            const uint32_t f = vn.w & 255u;
            const int32_t tk = (int32_t)vn.x;
            const uint32_t nx = vn.y;
            const uint32_t isw = f & F_WORM, isv = isw ^ 1u;
            const int32_t pos = 2 * tk + (int32_t)isw;
            occs += stt * (pos - lastp);
            lastp = pos;
            // the interval below a vertex ends here; a worm writes the same
            // slot, which the next vertex or the top of the slab overwrites
            qi[nq < qmax ? nq : qmax - 1] = ((uint32_t)(tk - ilo) << 1) | par;
            nq += (int)isv;
            nws += (int)isw;
            const uint32_t own_v = isv & (((f >> 1) & 3u) < 2u ? 1u : 0u);
            nvs += (int)own_v;
            nks += (int)(own_v & ((((f >> 3) & 1u) != (uint32_t)stt) ? 1u : 0u));
            ilo = isv ? tk : ilo;
            par = isv ? 0u : (par ^ 1u);
            stt = (int)((f >> 3) & 1u);
            if (j < capc) P.ev[ebase + (long long)j * nloc] = make_uint2((uint32_t)tk, f & 15u);
            j++;
            node = nx;
        }
        occ += occs;
        nv += nvs;
        nkink += nks;
        nwc += nws;
        if (j > capc) bad = true;
        P.cnt[cnt_base + s] = j > capc ? capc : j;
    }
    if (bad) atomicOr(&P.flags[chain], FL_OVERFLOW);
    __syncthreads();
    // terms of the improved estimator: l tanh(lambda l) for an even number
    // of worms in the interval, l / tanh(lambda l) for an odd number (one
    // division each; empty slots hold l = 0 and add nothing)
    double qimp = 0.0;
#pragma unroll 2
    for (int i = lane; i < NN; i += 64) {
        const uint32_t q = qint[i];
        const long long ell = (long long)(q >> 1);
        const double m = em1(sE, ell);
        const double num = m * (2.0 + m), den = 2.0 * (1.0 + m) + m * m;
        // the operands selected first: one division, and no branch that
        // would run both divisions for a mix of parities
        const bool odd = (q & 1u) != 0u;
        const double term = (double)ell * ((odd ? den : num) / (odd ? num : den));
        qimp += ell > 0 ? term : 0.0;
    }
    for (int o = 32; o > 0; o >>= 1) {
        nv += __shfl_down(nv, o, 64);
        nkink += __shfl_down(nkink, o, 64);
        nwc += __shfl_down(nwc, o, 64);
        occ += __shfl_down(occ, o, 64);
        qimp += __shfl_down(qimp, o, 64);
    }
    if (lane == 0) {
        DomPart dp;
        dp.nv = nv; dp.nkink = nkink; dp.nw = nwc; dp.occ2 = occ; dp.qimp = qimp; dp.windows = windows;
        P.dpart[C.dom_off + D] = dp;
    }
}

// The LDS form of one domain (12-byte nodes, see LdsStore).  `mem` is the
// LDS after the fixed region, `bytes` long.  Returns false, having written
// nothing outside LDS, when the domain's nodes or its worm list do not fit;
// the caller then takes the HBM store.
PMWA_DEV bool scatter_domain_lds(const Pools& P, const ChainDev& C, int chain, int D, unsigned char* mem,
                                 size_t bytes, uint64_t* __restrict__ ring, const int* __restrict__ off,
                                 const int* __restrict__ cnt, const uint64_t* __restrict__ sthr, int NE)
{
    const int lane = (int)threadIdx.x;
    const int k = D / C.ndsp, dsp = D - k * C.ndsp;
    const int nloc = C.nloc, ex = C.ex, ey = C.ey;
    const int NN = NE + 2 * nloc;
    const uint32_t BOT = (uint32_t)NE, TOP = (uint32_t)(NE + nloc);
    const uint16_t NIL = 0xFFFFu;
    const int32_t Tk = C.T[k], Tk1 = C.T[k + 1];
    // carve (arrays of an even length, so that each starts 4-byte aligned):
    // words, stamps, links, partner ends, then the worm list
    const size_t NNa = (size_t)((NN + 1) & ~1);
    const size_t nst = NNa / 2;
    const size_t fixed_b = NNa * 4 + nst * 4 + NNa * 6;
    if (NN >= 65535 || (long long)(Tk1 - Tk) >= (1LL << 27) || fixed_b + 64 > bytes) return false;
    const int wl_cap = (int)((bytes - fixed_b) / 2);
    LdsStore A;
    unsigned char* q = mem;
    A.w = reinterpret_cast<uint32_t*>(q); q += NNa * 4;
    A.own = reinterpret_cast<uint32_t*>(q); q += nst * 4;
    A.nxt = reinterpret_cast<uint16_t*>(q); q += NNa * 2;
    A.prv = reinterpret_cast<uint16_t*>(q); q += NNa * 2;
    A.aux = reinterpret_cast<uint16_t*>(q); q += NNa * 2;
    A.wl = reinterpret_cast<uint16_t*>(q);
    A.base = Tk;
    // Until the windows start, the stamps' memory (2 NN bytes) holds the
    // rank tables of the partner search: the node of every vertex, per site
    // (from off[s]) grouped by direction, then per site the vertex counts of
    // the four directions, 8 bits each.  The partner of the r-th vertex of
    // direction d on a site is the r-th vertex of direction d ^ 2 on the
    // neighbouring site (the two ends of a vertex carry the same tick).
    uint16_t* vnode = reinterpret_cast<uint16_t*>(A.own);
    uint32_t* dcnt = reinterpret_cast<uint32_t*>(vnode + NE + (NE & 1));

    // 1. nodes from the events (loads of consecutive sites are adjacent in
    //    HBM), the sentinels, the vertex counts per direction; vertices of
    //    bonds that leave the domain are marked as nodes a worm bounces off
    bool big = false;
    for (int s = lane; s < nloc; s += 64) {
        const int o = off[s], n = cnt[s];
        const int lx = s % ex, ly = s / ex;
        const uint32_t crm = ((C.dom_x > 1 && lx == ex - 1) ? 1u : 0u) | ((C.dom_y > 1 && ly == ey - 1) ? 2u : 0u) |
                             ((C.dom_x > 1 && lx == 0) ? 4u : 0u) | ((C.dom_y > 1 && ly == 0) ? 8u : 0u);
        const uint2* E = P.ev + ev_base(C, k, dsp, s);
        int c0 = 0, c1 = 0, c2 = 0, c3 = 0;
        for (int j0 = 0; j0 < n; j0 += 16) {
            uint2 e[16];
#pragma unroll
            for (int u = 0; u < 16; u++)
                if (j0 + u < n) e[u] = E[(long long)(j0 + u) * nloc];
#pragma unroll
            for (int u = 0; u < 16; u++) {
                const int j = j0 + u;
                if (j < n) {
                    const uint32_t idx = (uint32_t)(o + j);
                    const uint32_t f = e[u].y & 15u;
                    const uint32_t vd = (f >> 1) & 3u;
                    const bool v = (f & F_WORM) == 0u;
                    A.w[idx] = ((e[u].x - (uint32_t)Tk) << 5) | f | ((v && ((crm >> vd) & 1u)) ? F_SBOT : 0u);
                    A.prv[idx] = (uint16_t)(j > 0 ? idx - 1u : BOT + (uint32_t)s);
                    A.nxt[idx] = (uint16_t)(j + 1 < n ? idx + 1u : TOP + (uint32_t)s);
                    A.aux[idx] = NIL;
                    c0 += v && vd == 0u;
                    c1 += v && vd == 1u;
                    c2 += v && vd == 2u;
                    c3 += v && vd == 3u;
                }
            }
        }
        big |= (c0 | c1 | c2 | c3) > 255;
        dcnt[s] = (uint32_t)c0 | ((uint32_t)c1 << 8) | ((uint32_t)c2 << 16) | ((uint32_t)c3 << 24);
        const int bsv = P.bs[C.bs_off + unit_su(C, k, dsp, s)];
        A.w[BOT + s] = F_SBOT | (bsv ? F_UP : 0u);
        A.nxt[BOT + s] = (uint16_t)(n ? (uint32_t)o : TOP + s);
        A.prv[BOT + s] = NIL;
        A.aux[BOT + s] = NIL;
        A.w[TOP + s] = ((uint32_t)(Tk1 - Tk) << 5) | F_SBOT;
        A.prv[TOP + s] = (uint16_t)(n ? (uint32_t)(o + n - 1) : BOT + s);
        A.nxt[TOP + s] = NIL;
        A.aux[TOP + s] = NIL;
    }
    if (__any(big)) return false;          // a direction count beyond 8 bits: HBM store
    __syncthreads();
    // 2. vertex nodes by (site, direction, rank), and the worm list in
    //    (site, slot) order = node order
    int nw = 0;
    for (int base = 0; base < nloc; base += 64) {
        const int s = base + lane;
        uint32_t dc = 0;
        int ns = 0;
        if (s < nloc) {
            dc = dcnt[s];
            ns = cnt[s] - (int)((dc & 255u) + ((dc >> 8) & 255u) + ((dc >> 16) & 255u) + (dc >> 24));
        }
        int tot;
        int pos = nw + wave_excl_scan(ns, tot);
        if (s < nloc) {
            const int o = off[s], n = cnt[s];
            int r0 = 0, r1 = (int)(dc & 255u), r2 = r1 + (int)((dc >> 8) & 255u), r3 = r2 + (int)((dc >> 16) & 255u);
            for (int j0 = 0; j0 < n; j0 += 8) {
                uint32_t wb[8];
#pragma unroll
                for (int u = 0; u < 8; u++) wb[u] = j0 + u < n ? A.w[o + j0 + u] : 0u;
#pragma unroll
                for (int u = 0; u < 8; u++) {
                    if (j0 + u < n) {
                        const uint32_t idx = (uint32_t)(o + j0 + u);
                        const uint32_t vd = (wb[u] >> 1) & 3u;
                        if (wb[u] & F_WORM) {
                            if (pos < wl_cap) A.wl[pos] = (uint16_t)idx;
                            pos++;
                        } else {
                            const int r = vd == 0u ? r0 : vd == 1u ? r1 : vd == 2u ? r2 : r3;
                            vnode[o + r] = (uint16_t)idx;
                            r0 += vd == 0u;
                            r1 += vd == 1u;
                            r2 += vd == 2u;
                            r3 += vd == 3u;
                        }
                    }
                }
            }
        }
        nw += tot;
    }
    if (nw > wl_cap) return false;
    __syncthreads();
    // 3. partner ends: per site and direction (bonds inside the domain), the
    //    r-th vertex of direction d is matched with the r-th vertex of
    //    direction d ^ 2 on the neighbour (independent iterations)
    bool bad3 = false;
    for (int s = lane; s < nloc; s += 64) {
        const int o = off[s];
        const int lx = s % ex, ly = s / ex;
        const uint32_t dc = dcnt[s];
#pragma unroll
        for (int d = 0; d < 4; d++) {
            const bool cross = d == 0 ? (C.dom_x > 1 && lx == ex - 1) : d == 1 ? (C.dom_y > 1 && ly == ey - 1)
                             : d == 2 ? (C.dom_x > 1 && lx == 0) : (C.dom_y > 1 && ly == 0);
            if (cross) continue;
            const int nb = d == 0 ? (lx == ex - 1 ? s - (ex - 1) : s + 1)
                         : d == 1 ? (ly == ey - 1 ? s - (ey - 1) * ex : s + ex)
                         : d == 2 ? (lx == 0 ? s + (ex - 1) : s - 1)
                                  : (ly == 0 ? s + (ey - 1) * ex : s - ex);
            const int pd = d ^ 2;
            const uint32_t dn = dcnt[nb];
            int st = 0, nst_ = 0;
#pragma unroll
            for (int q = 0; q < 4; q++) {
                st += q < d ? (int)((dc >> (8 * q)) & 255u) : 0;
                nst_ += q < pd ? (int)((dn >> (8 * q)) & 255u) : 0;
            }
            const int nown = (int)((dc >> (8 * d)) & 255u), nnb = (int)((dn >> (8 * pd)) & 255u);
            bad3 |= nown != nnb;
            const int m_n = nown < nnb ? nown : nnb;
            const uint16_t* own_v = vnode + o + st;
            const uint16_t* nb_v = vnode + off[nb] + nst_;
#pragma unroll 4
            for (int r = 0; r < m_n; r++) {
                const uint32_t idx = own_v[r];
                const uint32_t m = nb_v[r];
                bad3 |= (A.w[idx] >> 5) != (A.w[m] >> 5);
                A.aux[idx] = (uint16_t)m;
            }
        }
    }
    if (bad3) atomicOr(&P.flags[chain], FL_STATE);
    __syncthreads();
    if (__any(P.flags[chain] != 0)) return true;

    // 4. N_cycle cycles, worms in list order, evaluated in windows
    for (int i = lane; i < (int)nst; i += 64) A.own[i] = 0u;
    __syncthreads();
    const long long windows = scatter_windows(A, ring, NN, nw, C, (uint32_t)P.sweep[chain], (uint32_t)D, sthr,
                                              &P.flags[chain]);

    // 5. measurement (Step 6) and write-back.  One lane per site follows the
    //    site's node list and writes the events back; the length and worm
    //    parity of every interval between vertices go to a table (in the
    //    memory of the previous-node and partner links, 4 NN bytes, which the
    //    walk does not read; site s has at most cnt[s] + 1 intervals, from
    //    slot off[s] + s), whose terms of the improved worm-density estimator
    //    all lanes then evaluate at once.
    __syncthreads();
    uint32_t* qint = reinterpret_cast<uint32_t*>(A.prv);
    for (int i = lane; i < NE + nloc; i += 64) qint[i] = 0u;
    __syncthreads();
    const int capc = C.cap;
    const long long cnt_base = C.cnt_off + unit_su(C, k, dsp, 0);
    const long long ev_base0 = ev_base(C, k, dsp, 0);
    long long nv = 0, nkink = 0, nwc = 0, occ = 0;
    bool bad = false;
    for (int s = lane; s < nloc; s += 64) {
        const long long ebase = ev_base0 + s;
        uint32_t* qi = qint + off[s] + s;
        const int qmax = cnt[s] + 1;
        int nq = 0;
        int stt = (int)((A.w[BOT + s] >> 3) & 1u);
        int32_t lastp = 2 * Tk;                 // positions in half ticks (< 2^31)
        int32_t ilo = Tk;
        uint32_t par = 0;
        int j = 0;
        uint32_t node = A.nxt[BOT + s];
        int guard = 0;
        int occs = 0, nvs = 0, nks = 0, nws_ = 0;
        for (;;) {
            if (node == TOP + (uint32_t)s) {
                occs += stt * (2 * Tk1 - lastp);
                if (nq < qmax) qi[nq] = ((uint32_t)(Tk1 - ilo) << 1) | par;
                else bad = true;
                break;
            }
            if (node >= (uint32_t)NE || ++guard > NE) { bad = true; break; }
            const NodeRec r = A.rec(node);
            const uint32_t f = r.f;
            const int32_t tk = r.t;
            const uint32_t nx = A.nxt[node];
            const uint32_t isw = f & F_WORM, isv = isw ^ 1u;
            const int32_t pos = 2 * tk + (int32_t)isw;
            occs += stt * (pos - lastp);
            lastp = pos;
            // the interval below a vertex ends here; a worm writes the same
            // slot, which the next vertex or the top of the slab overwrites
            qi[nq < qmax ? nq : qmax - 1] = ((uint32_t)(tk - ilo) << 1) | par;
            nq += (int)isv;
            nws_ += (int)isw;
            const uint32_t own_v = isv & (((f >> 1) & 3u) < 2u ? 1u : 0u);
            nvs += (int)own_v;
            nks += (int)(own_v & ((((f >> 3) & 1u) != (uint32_t)stt) ? 1u : 0u));
            ilo = isv ? tk : ilo;
            par = isv ? 0u : (par ^ 1u);
            stt = (int)((f >> 3) & 1u);
            if (j < capc) P.ev[ebase + (long long)j * nloc] = make_uint2((uint32_t)tk, f & 15u);
            j++;
            node = nx;
        }
        occ += occs;
        nv += nvs;
        nkink += nks;
        nwc += nws_;
        if (j > capc) bad = true;
        P.cnt[cnt_base + s] = j > capc ? capc : j;
    }
    if (bad) atomicOr(&P.flags[chain], FL_OVERFLOW);
    __syncthreads();
    // terms of the improved estimator: l tanh(lambda l) for an even number
    // of worms in the interval, l / tanh(lambda l) for an odd number (empty
    // slots hold l = 0 and add nothing); the expm1 table is read from L2
    const double* F = C.F;
    double qimp = 0.0;
#pragma unroll 4
    for (int i = lane; i < NE + nloc; i += 64) {
        const uint32_t q = qint[i];
        const long long ell = (long long)(q >> 1);
        const double m = em1(F, ell);
        const double num = m * (2.0 + m), den = 2.0 * (1.0 + m) + m * m;
        const bool odd = (q & 1u) != 0u;
        const double term = (double)ell * ((odd ? den : num) / (odd ? num : den));
        qimp += ell > 0 ? term : 0.0;
    }
    for (int o = 32; o > 0; o >>= 1) {
        nv += __shfl_down(nv, o, 64);
        nkink += __shfl_down(nkink, o, 64);
        nwc += __shfl_down(nwc, o, 64);
        occ += __shfl_down(occ, o, 64);
        qimp += __shfl_down(qimp, o, 64);
    }
    if (lane == 0) {
        DomPart dp;
        dp.nv = nv; dp.nkink = nkink; dp.nw = nwc; dp.occ2 = occ; dp.qimp = qimp; dp.windows = windows;
        P.dpart[C.dom_off + D] = dp;
    }
    return true;
}

// Dynamic LDS of the LDS form (HBM_ONLY = false): [exit thresholds 256 x u64]
// [ring 512 words][expm1 table 1024 doubles][off nloc+1][cnt nloc][nodes:
// tick 4B, nxt, prv, aux, wl 2B each, owner stamp 4B, fl 1B].  A domain whose
// nodes do not fit takes the HBM node store.
// The HBM form (HBM_ONLY = true) keeps only the thresholds and the ring in
// LDS (6 KB, so that as many wavefronts share a CU as their registers allow):
// the per-site counts and offsets go to the domain's scratch row in device
// memory, the expm1 table is read from the chain record (L2), every domain's
// nodes are in HBM.
template <bool HBM_ONLY>
__global__ void __launch_bounds__(64) k_scatter(Pools P, const int2* __restrict__ blk)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int2 bt = blk[blockIdx.x];
    const ChainDev& C = P.cd[bt.x];
    const int D = bt.y;
    const int lane = (int)threadIdx.x;
    if (D >= C.ntau * C.ndsp) return;
    const int k = D / C.ndsp, dsp = D - k * C.ndsp;
    const int nloc = C.nloc;
    uint64_t* sthr = reinterpret_cast<uint64_t*>(smem);
    uint64_t* ring = reinterpret_cast<uint64_t*>(smem + 256 * sizeof(uint64_t));
    const double* sE = C.F;
    int* off;
    if constexpr (HBM_ONLY) off = P.s_oc + C.oc_off + (long long)D * (2 * nloc + 2);
    else off = reinterpret_cast<int*>(smem + 768 * sizeof(uint64_t));
    int* cnt = off + (nloc + 1);
    // exit-leg thresholds ceil(P 2^53) of the cumulative scattering table
    // (exact: a power-of-two scaling, then an integral value below 2^55)
#pragma unroll
    for (int q = 0; q < 4; q++) sthr[q * 64 + lane] = (uint64_t)ceil(C.scat[q * 64 + lane] * 0x1.0p53);
    for (int s = lane; s < nloc; s += 64) cnt[s] = P.cnt[C.cnt_off + unit_su(C, k, dsp, s)];
    __syncthreads();
    // exclusive scan of the per-site counts
    int carry = 0;
    for (int base = 0; base < nloc; base += 64) {
        const int s = base + lane;
        const int v = s < nloc ? cnt[s] : 0;
        int tot;
        const int ex = wave_excl_scan(v, tot);
        if (s < nloc) off[s] = carry + ex;
        carry += tot;
    }
    if (lane == 0) off[nloc] = carry;
    __syncthreads();
    const int NE = carry;
    const int NN = NE + 2 * nloc;
    if (!live(P, C, bt.x)) return;

    if constexpr (!HBM_ONLY) {
        const size_t fixed = 768 * sizeof(uint64_t) + (size_t)(2 * nloc + 1) * sizeof(int);
        const size_t fixed_al = (fixed + 15) & ~(size_t)15;
        if ((size_t)P.lds_bytes > fixed_al &&
            scatter_domain_lds(P, C, bt.x, D, smem + fixed_al, (size_t)P.lds_bytes - fixed_al, ring, off, cnt, sthr,
                               NE))
            return;
    }
    if (NN > C.scr_nodes) { if (lane == 0) atomicOr(&P.flags[bt.x], FL_OVERFLOW); return; }
    const long long b = C.scr_off + (long long)D * C.scr_nodes;
    HbmStore A;
    A.nd = P.s_nd + b;
    A.wl = P.s_wl + b;
    A.own = P.s_own + b;
    A.stp = A.own;
    A.sh = 0;
    bool restore_oc = false;
    if constexpr (!HBM_ONLY) {
        // the owner stamps, the store's most frequent random accesses, stay
        // in the block's LDS when one per node pair fits there: after the
        // exit thresholds and the ring, over the per-site counts and offsets,
        // which the windows do not read (they are rebuilt after them)
        const size_t base = 768 * sizeof(uint64_t);
        if ((size_t)P.lds_bytes >= base + (size_t)((NN + 1) >> 1) * sizeof(uint32_t)) {
            A.stp = reinterpret_cast<uint32_t*>(smem + base);
            A.sh = 1;
            restore_oc = true;
        }
    }
    scatter_domain(P, C, bt.x, D, A, ring, off, cnt, sthr, sE, NE, restore_oc);
}
template __global__ void k_scatter<false>(Pools, const int2* __restrict__);
template __global__ void k_scatter<true>(Pools, const int2* __restrict__);

// ===========================================================================
// Boundary updates on the global arrays
// ===========================================================================
struct SiteArr {
    uint2* e;
    int st, n, cap;
    PMWA_DEV uint2 get(int j) const { return e[(long long)j * st]; }
    PMWA_DEV void put(int j, uint2 v) { e[(long long)j * st] = v; }
    // resize the range [lo, hi) to m entries (contents of the new range
    // undefined), moving the events above it.  They move 32 at a time: a
    // chunk's loads (from positions clamped to the events that move) are all
    // issued before its stores, so one round trip to memory serves the chunk,
    // and no chunk stores over an event that a later chunk still loads.  (A
    // chunk after the first waits for the earlier stores: loads and stores
    // share one counter of outstanding vector memory operations.)
    PMWA_DEV bool resize(int lo, int hi, int m)
    {
        constexpr int MB = 32;
        const int delta = m - (hi - lo);
        if (n + delta > cap) return false;
        if (delta > 0) {
            for (int top = n - 1; top >= hi; top -= MB) {
                uint2 v[MB];
#pragma unroll
                for (int q = 0; q < MB; q++) v[q] = get(top - q >= hi ? top - q : hi);
#pragma unroll
                for (int q = 0; q < MB; q++)
                    if (top - q >= hi) put(top - q + delta, v[q]);
            }
        } else if (delta < 0) {
            for (int b = hi; b < n; b += MB) {
                uint2 v[MB];
#pragma unroll
                for (int q = 0; q < MB; q++) v[q] = get(b + q < n ? b + q : n - 1);
#pragma unroll
                for (int q = 0; q < MB; q++)
                    if (b + q < n) put(b + q + delta, v[q]);
            }
        }
        n += delta;
        return true;
    }
};

// the sorted slots of an interval's worms: one or two in registers, more in
// the .x words of a column of event slots (tmp, stride st)
struct Slots {
    int n = 0;
    int32_t r0 = 0, r1 = 0;
    uint64_t dirs = 0;
    const uint2* tmp = nullptr;
    long long st = 0;
    PMWA_DEV int32_t off(int w) const { return n > 2 ? (int32_t)tmp[w * st].x : (w == 0 ? r0 : r1); }
};

// the slots of n worms on an interval of ell slots: registers for n <= 2,
// else the column at tmp.  False on failure (flagged).
template <class RS>
PMWA_DEV bool draw_slots(RS& rs, long long ell, int n, uint2* tmp, long long st, Slots& S, unsigned int* flag)
{
    S.n = n;
    S.tmp = tmp;
    S.st = st;
    if (n > 2) return worm_slots_col(rs, ell, n, EvCol{tmp, st}, S.dirs, flag);
    if (n > 0) return worm_slots_reg(rs, ell, n, S.r0, S.r1, S.dirs, flag);
    return true;
}

// writes the worms of an interval (slot base + offset, direction bit w of
// dirs) as events from position j0, occupation starting at p
PMWA_DEV void put_worms(SiteArr& A, int j0, int32_t base, const Slots& S, int p)
{
    int s = p;
    for (int w = 0; w < S.n; w++) {
        s ^= 1;
        A.put(j0 + w, make_uint2((uint32_t)(base + S.off(w)),
                                 1u | ((uint32_t)((S.dirs >> w) & 1u) << 1) | ((uint32_t)s << 3)));
    }
}

// Step 1, Eq. (Para): one lane per site, temporal boundaries k = 0.. in order;
// the upper domain's stream (site, k) makes the choice, then the worms of the
// two legs I_1 (above) and I_2 (below) are regenerated.
template <int LANES>
__global__ void __launch_bounds__(LANES) k_btemporal(Pools P, const int2* __restrict__ blk)
{
    const int2 bt = blk[blockIdx.x];
    const ChainDev& C = P.cd[bt.x];
    const int u = bt.y + (int)threadIdx.x;
    // the expm1 table is read from L2 (an LDS copy would take 8 KB more per
    // group and leave fewer groups per CU); worm slots go to registers or to
    // free event slots, not to LDS
    const double* sE = C.F;
    // the boundary ticks in LDS and the chain fields the loop reads in
    // registers: the loop's event stores could alias fields of C, which
    // would then be read again, after waiting for the stores, at every use
    __shared__ int32_t sT[NT_MAX + 1];
    for (int i = (int)threadIdx.x; i <= C.ntau; i += LANES) sT[i] = C.T[i];
    __syncthreads();
    if (u >= C.N || !live(P, C, bt.x)) return;
    const int nloc = C.nloc, cap = C.cap, ndsp = C.ndsp;
    const int32_t Mt = C.M;
    const uint32_t key0 = C.key0, key1 = C.key1, cid = C.chain_id;
    const long long ev_off = C.ev_off, cnt_off = C.cnt_off, bs_off = C.bs_off;
    auto usu = [&](int kk, int dd, int ss) { return (long long)(kk * ndsp + dd) * nloc + ss; };
    auto evb = [&](int kk, int dd, int ss) { return ev_off + (long long)(kk * ndsp + dd) * cap * nloc + ss; };
    unsigned int* flag = &P.flags[bt.x];
    const double lambda = C.lambda;
    const int dsp = u / C.nloc, sl = u % C.nloc;
    const int site = site_join(C, dsp, sl);
    const int nt = C.ntau;
    const uint32_t sweep = (uint32_t)P.sweep[bt.x];
    for (int k = 0; k < nt; k++) {
        Stream rs;
        rs.init_keys(key0, key1, cid, sweep, RNG_BT, (uint32_t)((long long)site * nt + k));
        const long long cuk = cnt_off + usu(k, dsp, sl);
        SiteArr Ak{P.ev + evb(k, dsp, sl), nloc, P.cnt[cuk], cap};
        uint8_t* sk = &P.bs[bs_off + usu(k, dsp, sl)];
        if (nt == 1) {
            bool hasv = false;
            for (int j = 0; j < Ak.n; j++) hasv |= !ev_worm(Ak.get(j).y);
            if (!hasv) {
                // the circle is one interval through the boundary
                const double W[2] = {1.0, 1.0};
                const int sp = choose(W, u53(rs.next()));
                const int m = worm_count(sE, lambda, rs, Mt, 0, flag);
                if (m < 0) return;
                // every event is replaced: the slots are drawn where the
                // worms go
                if (!Ak.resize(0, Ak.n, m)) { atomicOr(flag, FL_OVERFLOW); return; }
                Slots S1;
                if (!draw_slots(rs, Mt, m, Ak.e, nloc, S1, flag)) return;
                put_worms(Ak, 0, 0, S1, sp);
                P.cnt[cuk] = Ak.n;
                *sk = (uint8_t)sp;
                continue;
            }
        }
        // I_1: boundary up to the first vertex of slab k
        int jv = 0;
        while (jv < Ak.n && ev_worm(Ak.get(jv).y)) jv++;
        int32_t t1;
        int q;
        if (jv < Ak.n) { t1 = (int32_t)Ak.get(jv).x; q = jv > 0 ? (int)ev_up(Ak.get(jv - 1).y) : (int)*sk; }
        else { t1 = sT[k + 1]; q = P.bs[bs_off + usu((k + 1) % nt, dsp, sl)]; }
        const long long l1 = (long long)t1 - sT[k];
        // I_2: last vertex of slab k-1 up to the boundary
        const int kp = (k + nt - 1) % nt;
        const long long cukp = cnt_off + usu(kp, dsp, sl);
        SiteArr Bk{P.ev + evb(kp, dsp, sl), nloc, P.cnt[cukp], cap};
        int jl = Bk.n - 1;
        while (jl >= 0 && ev_worm(Bk.get(jl).y)) jl--;
        int32_t t2;
        int p;
        if (jl >= 0) { t2 = (int32_t)Bk.get(jl).x; p = (int)ev_up(Bk.get(jl).y); }
        else { t2 = sT[kp]; p = P.bs[bs_off + usu(kp, dsp, sl)]; }
        const long long l2 = (long long)sT[kp + 1] - t2;
        double W[2];
        for (int sp = 0; sp < 2; sp++) W[sp] = fleg(sE, sp ^ q, l1) * fleg(sE, p ^ sp, l2);
        const int sp = choose(W, u53(rs.next()));
        // each leg's count, then its slots.  More than two slots wait in the
        // top event slots of the leg's array (leg I_2's below leg I_1's when
        // there is one array); the resizes then keep the array below them
        // (a capacity that much smaller, while they are held)
        const int m1 = worm_count(sE, lambda, rs, l1, sp ^ q, flag);
        if (m1 < 0) return;
        const int h1 = m1 > 2 ? m1 : 0;
        if (Ak.n + h1 > cap) { atomicOr(flag, FL_OVERFLOW); return; }
        Slots S1, S2;
        if (!draw_slots(rs, l1, m1, Ak.e + (long long)(cap - h1) * nloc, nloc, S1, flag)) return;
        const int m2 = worm_count(sE, lambda, rs, l2, p ^ sp, flag);
        if (m2 < 0) return;
        const int h2 = m2 > 2 ? m2 : 0;
        if (nt == 1) {
            // same array: suffix first, then prefix
            if (Ak.n + h1 + h2 > cap) { atomicOr(flag, FL_OVERFLOW); return; }
            if (!draw_slots(rs, l2, m2, Ak.e + (long long)(cap - h1 - h2) * nloc, nloc, S2, flag)) return;
            Ak.cap = cap - h1 - h2;
            if (!Ak.resize(jl + 1, Ak.n, m2)) { atomicOr(flag, FL_OVERFLOW); return; }
            put_worms(Ak, jl + 1, t2, S2, p);
            if (!Ak.resize(0, jv, m1)) { atomicOr(flag, FL_OVERFLOW); return; }
            put_worms(Ak, 0, sT[k], S1, sp);
            P.cnt[cuk] = Ak.n;
        } else {
            if (Bk.n + h2 > cap) { atomicOr(flag, FL_OVERFLOW); return; }
            if (!draw_slots(rs, l2, m2, Bk.e + (long long)(cap - h2) * nloc, nloc, S2, flag)) return;
            Ak.cap = cap - h1;
            Bk.cap = cap - h2;
            if (!Ak.resize(0, jv, m1) || !Bk.resize(jl + 1, Bk.n, m2)) { atomicOr(flag, FL_OVERFLOW); return; }
            put_worms(Ak, 0, sT[k], S1, sp);
            put_worms(Bk, jl + 1, t2, S2, p);
            P.cnt[cuk] = Ak.n;
            P.cnt[cukp] = Bk.n;
        }
        *sk = (uint8_t)sp;
    }
}
template __global__ void k_btemporal<64>(Pools, const int2* __restrict__);
template __global__ void k_btemporal<16>(Pools, const int2* __restrict__);

// Step 2, Eq. (ParaSpace): one wavefront per (bond crossing a spatial domain
// boundary in direction d, slab); the bond is owned by the left/lower
// domain.  The bond's vertices in the slab are updated in tick order: a heat
// bath over the six allowed root states with the leg weights f, then the
// worms of the four legs are regenerated.
//
// Leg lengths and the occupations at the upper leg ends are fixed before the
// update starts (ticks never move; a vertex above is updated later), and the
// occupation at the lower end of a leg is either fixed or, when the previous
// vertex on that site is the bond's previous vertex, its new root.  So the
// wave computes, for every vertex in parallel, the choice for each of the
// four possible lower-end occupations, then follows the short chain of
// choices; worms are drawn per (vertex, leg) from their own streams, only
// for the legs that no later vertex regenerates, and both site arrays are
// rebuilt by prefix sums.  The result equals the vertices updated one by one.

// index of the previous / next vertex (worms skipped) for every position of
// a site array, by wave ballots (chunks of 64 with a carry)
PMWA_DEV void vertex_links(const uint2* A, int n, int16_t* pv, int16_t* nv)
{
    const int lane = (int)threadIdx.x;
    int carry = -1;
    for (int base = 0; base < n; base += 64) {
        const int j = base + lane;
        const bool v = j < n && !ev_worm(A[j].y);
        const unsigned long long m = __ballot(v);
        const unsigned long long below_m = m & ((1ULL << lane) - 1ULL);
        if (j < n) pv[j] = (int16_t)(below_m ? base + 63 - __clzll((long long)below_m) : carry);
        if (m) carry = base + 63 - __clzll((long long)m);
    }
    carry = n;
    for (int top = ((n + 63) / 64) * 64 - 64; top >= 0; top -= 64) {
        const int j = top + lane;
        const bool v = j < n && !ev_worm(A[j].y);
        const unsigned long long m = __ballot(v);
        const unsigned long long above_m = lane == 63 ? 0ULL : (m & ~((2ULL << lane) - 1ULL));
        if (j < n) nv[j] = (int16_t)(above_m ? top + __ffsll((long long)above_m) - 1 : carry);
        if (m) carry = top + __ffsll((long long)m) - 1;
    }
    __builtin_amdgcn_wave_barrier();
}

// positions of the vertices of direction `dir` in order: V[ord] = j and
// ord_of[j] = ord; returns their number
PMWA_DEV int bond_vertices(const uint2* A, int n, uint32_t dir, int* V, int16_t* ord_of, int vcap)
{
    const int lane = (int)threadIdx.x;
    int cnt = 0;
    for (int base = 0; base < n; base += 64) {
        const int j = base + lane;
        bool bv = false;
        if (j < n) {
            const uint2 e = A[j];
            bv = !ev_worm(e.y) && ev_dir(e.y) == dir;
        }
        const unsigned long long m = __ballot(bv);
        if (bv) {
            const int o = cnt + __popcll(m & ((1ULL << lane) - 1ULL));
            if (o < vcap) V[o] = j;
            ord_of[j] = (int16_t)o;
        }
        cnt += __popcll(m);
    }
    __builtin_amdgcn_wave_barrier();
    return cnt;
}

// wave-inclusive prefix sum of one int per lane
PMWA_DEV int wave_incl_sum(int x)
{
    const int lane = (int)threadIdx.x;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    return x;
}

// new array of one site: old vertices (bond vertices with new roots) and the
// worms of the intervals no bond vertex touches, plus the new worms; the new
// worms of interval (j, next vertex) start at pos[j] + 1 (or 0 for the
// interval below the first vertex).  Returns the new length.
PMWA_DEV int rebuild_positions(const uint2* A, int n, const int16_t* pv, const int16_t* nv, const int16_t* ord_of,
                               const BsVert* VV, uint32_t dir, int lower_leg, int upper_leg, int16_t* pos)
{
    const int lane = (int)threadIdx.x;
    auto is_bv = [&](int j) { return j >= 0 && j < n && !ev_worm(A[j].y) && ev_dir(A[j].y) == dir; };
    // worms inserted below the first vertex
    int first = n;
    if (n > 0) first = ev_worm(A[0].y) ? nv[0] : 0;
    int ins0 = 0;
    if (first < n && is_bv(first)) ins0 = VV[ord_of[first]].cnt[lower_leg];
    int carry = ins0;
    for (int base = 0; base < n; base += 64) {
        const int j = base + lane;
        int x = 0;
        if (j < n) {
            const uint2 e = A[j];
            if (!ev_worm(e.y)) {
                x = 1;
                const int u = nv[j];
                if (u < n && is_bv(u)) x += VV[ord_of[u]].cnt[lower_leg];
                else if (ev_dir(e.y) == dir) x += VV[ord_of[j]].cnt[upper_leg];
            } else {
                const int lo = pv[j], u = nv[j];
                const bool touched = is_bv(lo) || is_bv(u);
                x = touched ? 0 : 1;
            }
        }
        const int incl = wave_incl_sum(x);
        if (j < n) pos[j] = (int16_t)(carry + incl - x);
        carry += __shfl(incl, 63, 64);
    }
    __builtin_amdgcn_wave_barrier();
    return carry;
}

// copies the kept objects of A to their new positions in the site's event
// array O (stride st; bond vertices get their new occupation above)
PMWA_DEV void rebuild_copy(const uint2* A, int n, const int16_t* pv, const int16_t* nv, const int16_t* ord_of,
                           const BsVert* VV, uint32_t dir, int side, const int16_t* pos, uint2* O, long long st)
{
    const int lane = (int)threadIdx.x;
    auto is_bv = [&](int j) { return j >= 0 && j < n && !ev_worm(A[j].y) && ev_dir(A[j].y) == dir; };
    for (int j = lane; j < n; j += 64) {
        uint2 e = A[j];
        if (!ev_worm(e.y)) {
            if (ev_dir(e.y) == dir) {
                const uint32_t S = VV[ord_of[j]].S;
                const uint32_t up = side == 0 ? (S >> 2) & 1u : S >> 3;
                e.y = (e.y & ~8u) | (up << 3);
            }
            O[(long long)pos[j] * st] = e;
        } else if (!is_bv(pv[j]) && !is_bv(nv[j])) {
            O[(long long)pos[j] * st] = e;
        }
    }
}

// dynamic LDS (cap = event capacity):
//   A, B                   2 x cap uint2 (the rebuilt lists go straight to
//                          the event arrays in device memory)
//   pvA nvA ordA posA, the same for B      8 x cap int
//   VA, VB                  2 x cap int
//   VV                      cap BsVert
//   a pool of RW_POOL worm offsets (the lanes' offsets placed by a prefix
//   sum of their counts, in rounds if they need more)
// The expm1 table is read from global memory (it stays in L2).
__global__ void __launch_bounds__(64) k_bspatial(Pools P, const int2* __restrict__ blk, int d)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int2 bt = blk[blockIdx.x];
    const ChainDev& C = P.cd[bt.x];
    const int nt = C.ntau;
    const int u = bt.y / nt, k = bt.y % nt;   // cross bond, slab
    const int lane = (int)threadIdx.x;
    const int nb_units = d == 0 ? (C.dom_x > 1 ? C.Ly * C.dom_x : 0) : (C.dom_y > 1 ? C.Lx * C.dom_y : 0);
    if (u >= nb_units || !live(P, C, bt.x)) return;
    unsigned int* flag = &P.flags[bt.x];
    int a;
    if (d == 0) { const int y = u / C.dom_x, dx = u % C.dom_x; a = y * C.Lx + dx * C.ex + C.ex - 1; }
    else { const int dy = u / C.Lx, x = u % C.Lx; a = (dy * C.ey + C.ey - 1) * C.Lx + x; }
    const int c = nbr(C, a, d);
    int dspa, sla, dspc, slc;
    site_split(C, a, dspa, sla);
    site_split(C, c, dspc, slc);
    const int cap = C.cap, capb = C.capb;
    const double* sE = C.F;
    // dynamic LDS: the two site lists (cap events each), 16-bit links, ranks
    // and new positions per event, then per vertex of the bond (at most the
    // bond buffer's capacity) its indices and record, then the worm-offset
    // pool
    uint2* A = reinterpret_cast<uint2*>(smem);
    uint2* B = A + cap;
    BsVert* VV = reinterpret_cast<BsVert*>(B + cap);
    int* VA = reinterpret_cast<int*>(VV + capb);
    int* VB = VA + capb;
    int32_t* pool = VB + capb;
    int16_t* pvA = reinterpret_cast<int16_t*>(pool + RW_POOL);
    int16_t* nvA = pvA + cap;
    int16_t* ordA = nvA + cap;
    int16_t* posA = ordA + cap;
    int16_t* pvB = posA + cap;
    int16_t* nvB = pvB + cap;
    int16_t* ordB = nvB + cap;
    int16_t* posB = ordB + cap;

    const long long cua = C.cnt_off + unit_su(C, k, dspa, sla);
    const long long cuc = C.cnt_off + unit_su(C, k, dspc, slc);
    const int na = P.cnt[cua], nb = P.cnt[cuc];
    {
        const uint2* GA = P.ev + ev_base(C, k, dspa, sla);
        const uint2* GB = P.ev + ev_base(C, k, dspc, slc);
        for (int j = lane; j < na; j += 64) A[j] = GA[(long long)j * C.nloc];
        for (int j = lane; j < nb; j += 64) B[j] = GB[(long long)j * C.nloc];
    }
    __syncthreads();
    const int nva = bond_vertices(A, na, (uint32_t)d, VA, ordA, capb);
    const int nvb = bond_vertices(B, nb, (uint32_t)(d + 2), VB, ordB, capb);
    if (nva != nvb) { if (lane == 0) atomicOr(flag, FL_STATE); return; }
    if (nva > capb) { if (lane == 0) atomicOr(flag, FL_OVERFLOW); return; }
    const int nbv = nva;
    if (nbv == 0) return;
    vertex_links(A, na, pvA, nvA);
    vertex_links(B, nb, pvB, nvB);
    __syncthreads();

    const int bsa = P.bs[C.bs_off + unit_su(C, k, dspa, sla)];
    const int bsc = P.bs[C.bs_off + unit_su(C, k, dspc, slc)];
    const int bsa1 = P.bs[C.bs_off + unit_su(C, (k + 1) % nt, dspa, sla)];
    const int bsc1 = P.bs[C.bs_off + unit_su(C, (k + 1) % nt, dspc, slc)];
    const int32_t Tk = C.T[k], Tk1 = C.T[k + 1];
    const uint32_t sweep = (uint32_t)P.sweep[bt.x];
    const uint32_t unit = (uint32_t)((2LL * a + d) * nt + k);
    double vwa[6];
    {
        const int AL[6] = {0, 5, 6, 9, 10, 15};
#pragma unroll
        for (int m = 0; m < 6; m++) vwa[m] = C.vw[AL[m]];
    }

    // ---- every vertex: legs, fixed occupations, the choice per (p1, p2)
    bool bad = false;
    for (int v = lane; v < nbv; v += 64) {
        const int ja = VA[v], jc = VB[v];
        const int32_t t = (int32_t)A[ja].x;
        bad |= (int32_t)B[jc].x != t;
        const int la = pvA[ja], ha = nvA[ja], lc = pvB[jc], hc = nvB[jc];
        BsVert Vv;
        Vv.t = t;
        Vv.lo_a = la >= 0 ? (int32_t)A[la].x : Tk;
        Vv.lo_c = lc >= 0 ? (int32_t)B[lc].x : Tk;
        const int32_t hi_a = ha < na ? (int32_t)A[ha].x : Tk1;
        const int32_t hi_c = hc < nb ? (int32_t)B[hc].x : Tk1;
        Vv.l[0] = t - Vv.lo_a; Vv.l[1] = t - Vv.lo_c; Vv.l[2] = hi_a - t; Vv.l[3] = hi_c - t;
        const int p1f = la >= 0 ? (int)ev_up(A[la].y) : bsa;
        const int p2f = lc >= 0 ? (int)ev_up(B[lc].y) : bsc;
        const int q1 = ha < na ? (int)ev_up(A[ha - 1].y) : bsa1;
        const int q2 = hc < nb ? (int)ev_up(B[hc - 1].y) : bsc1;
        const bool prev_a = la >= 0 && !ev_worm(A[la].y) && ev_dir(A[la].y) == (uint32_t)d;
        const bool prev_c = lc >= 0 && !ev_worm(B[lc].y) && ev_dir(B[lc].y) == (uint32_t)(d + 2);
        const bool next_a = ha < na && ev_dir(A[ha].y) == (uint32_t)d;
        const bool next_c = hc < nb && ev_dir(B[hc].y) == (uint32_t)(d + 2);
        Vv.fl = (uint32_t)p1f | ((uint32_t)p2f << 1) | ((uint32_t)q1 << 2) | ((uint32_t)q2 << 3) |
                ((uint32_t)prev_a << 4) | ((uint32_t)prev_c << 5) | ((uint32_t)next_a << 6) | ((uint32_t)next_c << 7);
        double f0[4], f1[4];
#pragma unroll
        for (int g = 0; g < 4; g++) {
            const double m = em1(sE, (long long)Vv.l[g]);
            const double dd = 2.0 * (1.0 + m);
            f0[g] = 1.0 + (m * m) / dd;
            f1[g] = (m * (2.0 + m)) / dd;
        }
        Stream rs;
        rs.init(C, sweep, RNG_BS, unit);
        rs.w = (uint32_t)v << 17;
        const double uu = u53(rs.next());
        uint32_t m4 = 0;
#pragma unroll
        for (int x = 0; x < 4; x++) {
            const int p1 = x & 1, p2 = x >> 1;
            double W[6];
#pragma unroll
            for (int m = 0; m < 6; m++) {
                const int S = m == 0 ? 0 : m == 1 ? 5 : m == 2 ? 6 : m == 3 ? 9 : m == 4 ? 10 : 15;
                const int s1 = S & 1, s2 = (S >> 1) & 1, s1p = (S >> 2) & 1, s2p = S >> 3;
                const double g0 = (p1 ^ s1) ? f1[0] : f0[0];
                const double g1 = (p2 ^ s2) ? f1[1] : f0[1];
                const double g2 = (s1p ^ q1) ? f1[2] : f0[2];
                const double g3 = (s2p ^ q2) ? f1[3] : f0[3];
                W[m] = (((g0 * g1) * g2) * g3) * vwa[m];
            }
            // an occupation pair with no allowed root pattern (zero-length
            // legs of the wrong parity) gets the marker 15; only the pair
            // the chain actually reaches is used, and it always has one
            m4 |= ((uint32_t)choose(W, uu) & 15u) << (4 * x);
        }
        Vv.m4 = m4;
        VV[v] = Vv;
    }
    if (__ballot(bad)) { if (lane == 0) atomicOr(flag, FL_STATE); return; }
    __syncthreads();

    // ---- the chain of choices (uniform on every lane)
    {
        int s1p_prev = 0, s2p_prev = 0;
        for (int v = 0; v < nbv; v++) {
            const uint32_t fl = VV[v].fl, m4 = VV[v].m4;
            const int p1 = (fl & 16u) ? s1p_prev : (int)(fl & 1u);
            const int p2 = (fl & 32u) ? s2p_prev : (int)((fl >> 1) & 1u);
            const int m = (int)((m4 >> (4 * (p1 | (p2 << 1)))) & 15u);
            const int S = m == 0 ? 0 : m == 1 ? 5 : m == 2 ? 6 : m == 3 ? 9 : m == 4 ? 10 : 15;
            if (lane == 0) {
                if (m > 5) atomicOr(flag, FL_STATE);
                VV[v].S = (uint32_t)S;
                VV[v].p12 = (uint32_t)(p1 | (p2 << 1));
            }
            s1p_prev = (S >> 2) & 1;
            s2p_prev = S >> 3;
        }
    }
    __syncthreads();

    // ---- worm counts of the legs that stay (lane per (vertex, leg))
    const double lambda = C.lambda;
    for (int w0 = 0; w0 < 4 * nbv; w0 += 64) {
        const int uvg = w0 + lane;
        if (uvg < 4 * nbv) {
            const int v = uvg >> 2, g = uvg & 3;
            const BsVert& Vv = VV[v];
            const bool dead = (g == 2 && (Vv.fl & 64u)) || (g == 3 && (Vv.fl & 128u));
            int n = 0;
            if (!dead) {
                const int S = (int)Vv.S, p1 = (int)(Vv.p12 & 1u), p2 = (int)(Vv.p12 >> 1);
                const int s1 = S & 1, s2 = (S >> 1) & 1, s1p = (S >> 2) & 1, s2p = S >> 3;
                const int q1 = (int)((Vv.fl >> 2) & 1u), q2 = (int)((Vv.fl >> 3) & 1u);
                const int sig = g == 0 ? p1 ^ s1 : g == 1 ? p2 ^ s2 : g == 2 ? s1p ^ q1 : s2p ^ q2;
                Stream rs;
                rs.init(C, sweep, RNG_BSL + (uint32_t)g, unit);
                rs.w = (uint32_t)v << 17;
                n = worm_count(sE, lambda, rs, (long long)Vv.l[g], sig, flag);
                if (n < 0) n = 0;
            }
            VV[v].cnt[g] = n;
        }
    }
    __syncthreads();

    // ---- new arrays: positions, kept objects, then the new worms
    const int na2 = rebuild_positions(A, na, pvA, nvA, ordA, VV, (uint32_t)d, 0, 2, posA);
    const int nb2 = rebuild_positions(B, nb, pvB, nvB, ordB, VV, (uint32_t)(d + 2), 1, 3, posB);
    if (na2 > cap || nb2 > cap) { if (lane == 0) atomicOr(flag, FL_OVERFLOW); return; }
    __syncthreads();
    // the new lists go straight to the sites' event arrays: their old
    // contents were copied to A and B at the start, and no other block reads
    // these two sites in this launch (the stride in a register, and both
    // addresses before the first store, which would otherwise make the
    // compiler reload them after it)
    const long long st = C.nloc;
    uint2* OA = P.ev + ev_base(C, k, dspa, sla);
    uint2* OB = P.ev + ev_base(C, k, dspc, slc);
    asm volatile("" ::"v"(OA), "v"(OB), "v"(st));
    rebuild_copy(A, na, pvA, nvA, ordA, VV, (uint32_t)d, 0, posA, OA, st);
    rebuild_copy(B, nb, pvB, nvB, ordB, VV, (uint32_t)(d + 2), 1, posB, OB, st);
    for (int w0 = 0; w0 < 4 * nbv; w0 += 64) {
        const int uvg = w0 + lane;
        int n = 0;
        if (uvg < 4 * nbv) n = VV[uvg >> 2].cnt[uvg & 3];
        // offsets through the pool; the first pending lane always fits
        // (n <= NWL < RW_POOL), so every round makes progress
        const int wst = wave_incl_sum(n) - n;
        bool todo = n > 0;
        for (unsigned long long pend = __ballot(todo); pend; pend = __ballot(todo)) {
            const int first = __ffsll((long long)pend) - 1;
            const int pb = __shfl(wst, first, 64);
            if (todo && wst + n <= pb + RW_POOL) {
                const int v = uvg >> 2, g = uvg & 3;
                const BsVert& Vv = VV[v];
                const int S = (int)Vv.S, p1 = (int)(Vv.p12 & 1u), p2 = (int)(Vv.p12 >> 1);
                const int s1 = S & 1, s2 = (S >> 1) & 1, s1p = (S >> 2) & 1, s2p = S >> 3;
                const int q1 = (int)((Vv.fl >> 2) & 1u), q2 = (int)((Vv.fl >> 3) & 1u);
                const int sig = g == 0 ? p1 ^ s1 : g == 1 ? p2 ^ s2 : g == 2 ? s1p ^ q1 : s2p ^ q2;
                const int start_occ = g == 0 ? p1 : g == 1 ? p2 : g == 2 ? s1p : s2p;
                const int32_t base = g == 0 ? Vv.lo_a : g == 1 ? Vv.lo_c : Vv.t;
                // first output slot: just above the leg's lower delimiter
                int at;
                if (g == 0) { const int lo = pvA[VA[v]]; at = lo >= 0 ? posA[lo] + 1 : 0; }
                else if (g == 1) { const int lo = pvB[VB[v]]; at = lo >= 0 ? posB[lo] + 1 : 0; }
                else if (g == 2) at = posA[VA[v]] + 1;
                else at = posB[VB[v]] + 1;
                uint2* O = (g == 0 || g == 2) ? OA : OB;
                // the count words again, then the slots (same stream)
                Stream rs;
                rs.init(C, sweep, RNG_BSL + (uint32_t)g, unit);
                rs.w = (uint32_t)v << 17;
                (void)worm_count(sE, lambda, rs, (long long)Vv.l[g], sig, flag);
                int32_t* o = pool + (wst - pb);
                uint64_t dirs;
                if (worm_slots<1>(rs, (long long)Vv.l[g], n, o, dirs, flag)) {
                    for (int w = 0; w < n; w++) {
                        const uint32_t occ = (uint32_t)((start_occ + w + 1) & 1);
                        O[(long long)(at + w) * st] =
                            make_uint2((uint32_t)(base + o[w]), 1u | ((uint32_t)((dirs >> w) & 1u) << 1) | (occ << 3));
                    }
                }
                todo = false;
            }
            __builtin_amdgcn_wave_barrier();
        }
    }
    if (lane == 0) { P.cnt[cua] = na2; P.cnt[cuc] = nb2; }
}

// ===========================================================================
// Step 4 with one wavefront per (site, slab): the entries of the four bond
// buffers are ranked in (tick, bond id) order by counting, every interval
// draws its worms from its own word range in parallel, and a prefix sum
// places the events.  Same result as k_assemble.
// dynamic LDS: val[nmax], merged val[nmax] (u32), a pool of RW_POOL worm
// offsets, slot[nmax], merged slot[nmax] (u8).  The intervals' worm counts
// are drawn first; a prefix sum over the wave places every lane's offsets in
// the pool, in rounds if the 64 intervals together have more than RW_POOL.
// ===========================================================================
__global__ void __launch_bounds__(64) k_assemble_w(Pools P, const int2* __restrict__ blk, int nmax)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int2 bt = blk[blockIdx.x];
    const ChainDev& C = P.cd[bt.x];
    const int u = bt.y;
    const int lane = (int)threadIdx.x;
    if (u >= C.ntau * C.N || !live(P, C, bt.x)) return;
    // merge keys (a multiple of 4 entries, 16-byte aligned), entries,
    // merged entries, the worm-offset pool, bond slots of both
    const int nmax4 = (nmax + 3) & ~3;
    uint32_t* keys = reinterpret_cast<uint32_t*>(smem);
    uint32_t* val = keys + nmax4;
    uint32_t* mval = val + nmax;
    int32_t* pool = reinterpret_cast<int32_t*>(mval + nmax);
    uint8_t* vsl = reinterpret_cast<uint8_t*>(pool + RW_POOL);
    uint8_t* msl = vsl + nmax;
    unsigned int* flag = &P.flags[bt.x];
    const int sl = u % C.nloc;
    const int rr = u / C.nloc;
    const int dsp = rr % C.ndsp, k = rr / C.ndsp;
    const int i = site_join(C, dsp, sl);
    const int st = C.nloc;
    uint2* E = P.ev + ev_base(C, k, dsp, sl);
    const long long cu = C.cnt_off + unit_su(C, k, dsp, sl);
    const int s_lo = P.bs[C.bs_off + unit_su(C, k, dsp, sl)];
    const int s_hi = P.bs[C.bs_off + unit_su(C, (k + 1) % C.ntau, dsp, sl)];
    long long bids[4];
    int base = 0;
#pragma unroll
    for (int d = 0; d < 4; d++) {
        const int a = (d < 2) ? i : nbr(C, i, d);
        int dspa, sla;
        site_split(C, a, dspa, sla);
        const int bd = d & 1;
        const long long row = (long long)((k * 2 + bd) * C.ndsp + dspa);
        const uint32_t* src = P.bv + C.bv_off + row * C.capb * C.nloc + sla;
        const int ns = P.bvc[C.bvc_off + row * C.nloc + sla];
        bids[d] = 2LL * a + bd;
        if (base + ns > nmax) { if (lane == 0) atomicOr(flag, FL_OVERFLOW); return; }
        for (int j = lane; j < ns; j += 64) {
            val[base + j] = src[(long long)j * st];
            vsl[base + j] = (uint8_t)d;
        }
        base += ns;
    }
    const int nv = base;
    __syncthreads();
    // merged order: (tick, bond id) keys of a site are distinct.  The four
    // bonds are ranked once (2 bits each in brk), so an entry's key is the
    // 32-bit 4 tick + rank of its bond (ticks are below 2^29)
    uint32_t brk = 0;
#pragma unroll
    for (int d = 0; d < 4; d++) {
        uint32_t r = 0;
#pragma unroll
        for (int d2 = 0; d2 < 4; d2++) r += bids[d2] < bids[d] ? 1u : 0u;
        brk |= r << (2 * d);
    }
    // every entry's key once (padding keys above all of them), then each
    // entry's rank among them, four keys per LDS read
    const int nv4 = (nv + 3) & ~3;
    for (int e = lane; e < nv4; e += 64)
        keys[e] = e < nv ? ((val[e] & BV_TICK) << 2) | ((brk >> (2 * (uint32_t)vsl[e])) & 3u) : 0xFFFFFFFFu;
    __syncthreads();
    const uint4* keys4 = reinterpret_cast<const uint4*>(keys);
    for (int e = lane; e < nv; e += 64) {
        const uint32_t key = keys[e];
        int rank = 0;
        for (int e4 = 0; e4 < nv4 / 4; e4++) {
            const uint4 q = keys4[e4];
            rank += (q.x < key ? 1 : 0) + (q.y < key ? 1 : 0) + (q.z < key ? 1 : 0) + (q.w < key ? 1 : 0);
        }
        mval[rank] = val[e];
        msl[rank] = vsl[e];
    }
    __syncthreads();
    // intervals r = 0..nv (below vertex r; the last one ends at T_k+1)
    const uint32_t sweep = (uint32_t)P.sweep[bt.x];
    const uint32_t unit = (uint32_t)((long long)i * C.ntau + k);
    // read before the event stores below, which could alias fields of C
    const int capw = C.cap;
    const int32_t Tk0 = C.T[k], Tk1 = C.T[k + 1];
    const double lambda = C.lambda;
    const int nint = nv + 1;
    int carry = 0;
    bool bad = false;
    for (int r0 = 0; r0 < nint; r0 += 64) {
        const int r = r0 + lane;
        int nwr = 0;
        int32_t lo = 0, hi = 0;
        int p = 0;
        bool has_v = false;
        uint32_t vinfo = 0;
        Stream rs;
        if (r < nint) {
            if (r > 0) {
                const uint32_t v = mval[r - 1];
                const uint32_t d = msl[r - 1];
                lo = (int32_t)(v & BV_TICK);
                const int qq = (int)((d < 2 ? v >> 30 : v >> 31) & 1u);
                p = qq ^ (int)((v >> 29) & 1u);
            } else {
                lo = Tk0;
                p = s_lo;
            }
            int q;
            if (r < nv) {
                const uint32_t v = mval[r];
                const uint32_t d = msl[r];
                hi = (int32_t)(v & BV_TICK);
                q = (int)((d < 2 ? v >> 30 : v >> 31) & 1u);
                const int above = q ^ (int)((v >> 29) & 1u);
                has_v = true;
                vinfo = (d << 1) | ((uint32_t)above << 3);
            } else {
                hi = Tk1;
                q = s_hi;
            }
            rs.init(C, sweep, RNG_R, unit);
            rs.w = (uint32_t)r << 17;
            nwr = worm_count(C.F, lambda, rs, (long long)hi - lo, p ^ q, flag);
            if (nwr < 0) { bad = true; nwr = 0; }
        }
        const int x = nwr + (has_v ? 1 : 0);
        const int incl = wave_incl_sum(x);
        const int pos = carry + incl - x;
        carry += __shfl(incl, 63, 64);
        const bool fits = r < nint && pos + x <= capw;
        // slots through the pool; the first pending lane always fits
        // (nwr <= NWL < RW_POOL), so every round makes progress
        const int wst = wave_incl_sum(nwr) - nwr;
        bool todo = nwr > 0;
        for (unsigned long long pend = __ballot(todo); pend; pend = __ballot(todo)) {
            const int first = __ffsll((long long)pend) - 1;
            const int pb = __shfl(wst, first, 64);
            if (todo && wst + nwr <= pb + RW_POOL) {
                int32_t* o = pool + (wst - pb);
                uint64_t dirs;
                if (!worm_slots<1>(rs, (long long)hi - lo, nwr, o, dirs, flag)) {
                    bad = true;
                } else if (fits) {
                    int sst = p;
                    for (int w = 0; w < nwr; w++) {
                        sst ^= 1;
                        E[(long long)(pos + w) * st] = make_uint2((uint32_t)(lo + o[w]),
                                                                  1u | ((uint32_t)((dirs >> w) & 1u) << 1) | ((uint32_t)sst << 3));
                    }
                }
                todo = false;
            }
            __builtin_amdgcn_wave_barrier();
        }
        if (has_v && fits) E[(long long)(pos + nwr) * st] = make_uint2((uint32_t)hi, vinfo);
    }
    if (__ballot(bad)) return;
    if (carry > capw) { if (lane == 0) atomicOr(flag, FL_OVERFLOW); return; }
    if (lane == 0) P.cnt[cu] = carry;
}

// ===========================================================================
// Green function of Q = b + b^+ on the current configuration (Supplemental
// S-I, n = 2): G(r, dt) = (1/N) sum_i <Q_i(tau) Q_{i+r}(tau + dt)>, averaged
// over tau.  The one-point ratio rho/eta on an interval (delimited by
// vertices and temporal domain boundaries) is tanh(lambda l) for an even
// number of worms in it and coth(lambda l) for an odd number; two points on
// different intervals give the product of their ratios, two points on one
// interval give 1 (Q commutes with the interval propagator, Q^2 = 1).
// One lane per (site i, slab k, displacement): the lane merges the
// intervals of site i in slab k with those of site i + r from the partner
// time T_k + dt on (across slabs, wrapping at beta).  Block
// (k * nd + d) * nchunk + c covers sites 64 c .. 64 c + 63 and writes the
// wave sum of its lanes to part[block].
// ===========================================================================
// sequential reader of one site's events in a slab, four loads at a time
struct EvReader {
    const uint2* E;
    int st, n, j, b;
    uint2 q0, q1, q2, q3;
    PMWA_DEV void init(const uint2* e, int stride, int cnt) { E = e; st = stride; n = cnt; j = 0; b = 4; }
    PMWA_DEV bool next(uint2& e)
    {
        if (j >= n) return false;
        if (b == 4) {
            const int base = j;
            q0 = E[(long long)base * st];
            if (base + 1 < n) q1 = E[(long long)(base + 1) * st];
            if (base + 2 < n) q2 = E[(long long)(base + 2) * st];
            if (base + 3 < n) q3 = E[(long long)(base + 3) * st];
            b = 0;
        }
        e = b == 0 ? q0 : b == 1 ? q1 : b == 2 ? q2 : q3;
        b++;
        j++;
        return true;
    }
};

// the interval that starts at tick `start`: its end (the next vertex, else
// the top of the slab) and its ratio g
PMWA_DEV void green_interval(EvReader& R, int32_t top, const double* __restrict__ F, int32_t start,
                             int32_t& end, double& g)
{
    uint32_t par = 0;
    uint2 e;
    end = top;
    while (R.next(e)) {
        if (e.y & 1u) { par ^= 1u; continue; }
        end = (int32_t)e.x;
        break;
    }
    const long long ell = (long long)end - start;
    g = 0.0;                           // an empty interval holds no worm
    if (ell > 0) {
        const double m = em1(F, ell);
        const double num = m * (2.0 + m), den = 2.0 * (1.0 + m) + m * m;
        g = par ? den / num : num / den;
    }
}

__global__ void __launch_bounds__(64) k_green(Pools P, int chain, const int4* __restrict__ disp, int nd,
                                              int nchunk, double* __restrict__ part)
{
    const ChainDev& C = P.cd[chain];
    const int lane = (int)threadIdx.x;
    const int blk = (int)blockIdx.x;
    const int c = blk % nchunk, kd = blk / nchunk;
    const int d = kd % nd, k = kd / nd;
    const int i = c * 64 + lane;
    const int4 r = disp[d];            // 0 <= r.x < Lx, 0 <= r.y < Ly, 0 <= r.z < M
    double acc = 0.0;
    if (i < C.N) {
        const int x = i % C.Lx, y = i / C.Lx;
        const int jj = ((y + r.y) % C.Ly) * C.Lx + (x + r.x) % C.Lx;
        int dspi, sli, dspj, slj;
        site_split(C, i, dspi, sli);
        site_split(C, jj, dspj, slj);
        const double* F = C.F;
        const int32_t M = C.M, nt = C.ntau;
        const int32_t Tk = C.T[k], Tk1 = C.T[k + 1];
        // site i, slab k
        EvReader A;
        A.init(P.ev + ev_base(C, k, dspi, sli), C.nloc, P.cnt[C.cnt_off + unit_su(C, k, dspi, sli)]);
        int32_t sa = Tk, ea;
        double ga;
        green_interval(A, Tk1, F, sa, ea, ga);
        // site jj from the partner time of T_k: its slab kb and interval
        int32_t pos = Tk + r.z;
        if (pos >= M) pos -= M;
        int kb = 0;
        while (C.T[kb + 1] <= pos) kb++;
        EvReader B;
        B.init(P.ev + ev_base(C, kb, dspj, slj), C.nloc, P.cnt[C.cnt_off + unit_su(C, kb, dspj, slj)]);
        int32_t sb = C.T[kb], eb;
        double gb;
        green_interval(B, C.T[kb + 1], F, sb, eb, gb);
        while (eb <= pos) {
            sb = eb;
            green_interval(B, C.T[kb + 1], F, sb, eb, gb);
        }
        int32_t tau = Tk;
        // every step closes an interval of one of the two sites: at most the
        // events of both sites over all slabs plus the slab ends (a bound
        // that only an inconsistent state could reach)
        int guard = 2 * (C.cap + 2) * (nt + 1);
        while (tau < Tk1 && --guard > 0) {
            int32_t len = ea - tau;
            const int32_t lb = eb - pos;
            if (lb < len) len = lb;
            if (len < 0) break;
            const bool same = jj == i && kb == k && sb == sa;
            acc += (double)len * (same ? 1.0 : ga * gb);
            tau += len;
            pos += len;
            if (tau >= Tk1) break;
            if (tau == ea) {
                sa = ea;
                green_interval(A, Tk1, F, sa, ea, ga);
            }
            if (pos == eb) {
                if (eb == C.T[kb + 1]) {
                    // next slab of site jj; past the last one time wraps at beta
                    kb++;
                    if (kb == nt) { kb = 0; pos -= M; }
                    B.init(P.ev + ev_base(C, kb, dspj, slj), C.nloc, P.cnt[C.cnt_off + unit_su(C, kb, dspj, slj)]);
                    sb = C.T[kb];
                } else {
                    sb = eb;
                }
                green_interval(B, C.T[kb + 1], F, sb, eb, gb);
            }
        }
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
    if (lane == 0) part[blk] = acc;
}

// ===========================================================================
// n-point functions of b, b^+ and Q (Supplemental S-I).  The worms of an
// interval (delimited by vertices and temporal domain boundaries) are summed
// over: an operator inserted on it multiplies its propagator element
// <q| E(l) |p> (E = exp(l eta Delta Q)) by the ratio
// <q| E .. O_m .. O_1 E |p> / <q| E |p>, operators in time order; points on
// different intervals give the product of their intervals' ratios.  A point
// at tick t sits at t + 1/4 (between a vertex at t and the worm slot
// t + 1/2).  One lane per (site, base time) of one correlator; block
// c * nchunk + b covers pairs 64 b .. 64 b + 63 of correlator c and writes
// the wave sum to part[block].
// ===========================================================================
constexpr int CORR_NPT = 8;

// the interval of `site` holding time t + 1/4: lo <= t < hi, the occupation
// p just above lo and q just below hi
PMWA_DEV void corr_interval(const Pools& P, const ChainDev& C, int site, int32_t t, int32_t& lo, int32_t& hi,
                            int& p, int& q)
{
    int kb = 0;
    while (C.T[kb + 1] <= t) kb++;
    int dsp, sl;
    site_split(C, site, dsp, sl);
    const long long su = unit_su(C, kb, dsp, sl);
    const int n = P.cnt[C.cnt_off + su];
    const uint2* E = P.ev + ev_base(C, kb, dsp, sl);
    int state = P.bs[C.bs_off + su];
    lo = C.T[kb];
    p = state;
    hi = C.T[kb + 1];
    q = P.bs[C.bs_off + unit_su(C, kb + 1 == C.ntau ? 0 : kb + 1, dsp, sl)];
    for (int j = 0; j < n; j++) {
        const uint2 e = E[(long long)j * C.nloc];
        const int up = (int)((e.y >> 3) & 1u);
        if (!(e.y & 1u)) {
            if ((int32_t)e.x <= t) { lo = (int32_t)e.x; p = up; }
            else { hi = (int32_t)e.x; q = state; break; }
        }
        state = up;
    }
}

__global__ void __launch_bounds__(64) k_corr(Pools P, int chain, const int4* __restrict__ pts, int npt, int nbase,
                                             int nchunk, double* __restrict__ part)
{
    const ChainDev& C = P.cd[chain];
    const int lane = (int)threadIdx.x;
    const int blk = (int)blockIdx.x;
    const int c = blk / nchunk, b = blk - c * nchunk;
    const long long u = (long long)b * 64 + lane;
    double acc = 0.0;
    if (u < (long long)C.N * nbase) {
        const int i = (int)(u / nbase), j = (int)(u - (long long)i * nbase);
        const int x = i % C.Lx, y = i / C.Lx;
        const int32_t tau = (int32_t)(((long long)j * C.M) / nbase);
        int site[CORR_NPT], op[CORR_NPT], pp[CORR_NPT], qq[CORR_NPT], grp[CORR_NPT];
        int32_t t[CORR_NPT], lo[CORR_NPT], hi[CORR_NPT];
        for (int k = 0; k < npt; k++) {
            const int4 r = pts[c * npt + k];        // 0 <= rx < Lx, 0 <= ry < Ly, 0 <= dt < M
            site[k] = ((y + r.y) % C.Ly) * C.Lx + (x + r.x) % C.Lx;
            int32_t tk = tau + r.z;
            if (tk >= C.M) tk -= C.M;
            t[k] = tk;
            op[k] = r.w;
            corr_interval(P, C, site[k], tk, lo[k], hi[k], pp[k], qq[k]);
            grp[k] = -1;
        }
        const double* F = C.F;
        double prod = 1.0;
        for (int k = 0; k < npt; k++) {
            if (grp[k] >= 0) continue;
            int mem[CORR_NPT], nm = 0;
            for (int m = k; m < npt; m++)
                if (site[m] == site[k] && lo[m] == lo[k] && hi[m] == hi[k]) {
                    grp[m] = k;
                    mem[nm++] = m;
                }
            // bottom to top: ascending time, at equal times the later-listed
            // point first (the first listed is leftmost)
            for (int a = 1; a < nm; a++) {
                const int v = mem[a];
                int bb = a - 1;
                while (bb >= 0 && (t[mem[bb]] > t[v] || (t[mem[bb]] == t[v] && mem[bb] < v))) {
                    mem[bb + 1] = mem[bb];
                    bb--;
                }
                mem[bb + 1] = v;
            }
            double v0 = pp[k] ? 0.0 : 1.0, v1 = pp[k] ? 1.0 : 0.0;
            int32_t cur = lo[k];
            for (int a = 0; a <= nm; a++) {
                const int32_t te = a < nm ? t[mem[a]] : hi[k];
                const long long ell = (long long)(te - cur);
                const double ch = fleg(F, 0, ell), sh = fleg(F, 1, ell);
                const double n0 = ch * v0 + sh * v1;
                const double n1 = sh * v0 + ch * v1;
                v0 = n0;
                v1 = n1;
                if (a < nm) {
                    const int o = op[mem[a]];
                    const double w0 = v0, w1 = v1;
                    if (o == 0) { v0 = w1; v1 = w0; }          // b + b^+
                    else if (o == 1) { v0 = w1; v1 = 0.0; }    // b:   |1> -> |0>
                    else { v0 = 0.0; v1 = w0; }                // b^+: |0> -> |1>
                    cur = te;
                }
            }
            const double den = fleg(F, pp[k] ^ qq[k], (long long)(hi[k] - lo[k]));
            prod = prod * ((qq[k] ? v1 : v0) / den);
        }
        acc = prod;
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
    if (lane == 0) part[blk] = acc;
}

// The per-block partials of k_green summed per displacement on the device,
// in the order the host sums them for pmwa_green (slab, then block of
// sites), then divided by M N: out[d] = G of displacement d.
__global__ void __launch_bounds__(64) k_green_sum(const double* __restrict__ part, int ntau, int nd, int nchunk,
                                                  double norm, double* __restrict__ out)
{
    const int d = (int)(blockIdx.x * 64 + threadIdx.x);
    if (d >= nd) return;
    double sum = 0.0;
    for (int k = 0; k < ntau; k++)
        for (int c = 0; c < nchunk; c++) sum += part[((long long)k * nd + d) * nchunk + c];
    out[d] = sum / norm;
}

// ===========================================================================
// End of sweep: per chain, sum the domain partials in domain order, append
// the record to the series ring, advance the sweep counter.
// ===========================================================================
__global__ void __launch_bounds__(256) k_finish(Pools P, const int* __restrict__ chains)
{
    const int chain = chains[blockIdx.x];
    const ChainDev& C = P.cd[chain];
    if (!live(P, C, chain)) return;
    const int nd = (int)C.n_dom;
    const int tid = (int)threadIdx.x;
    const int per = (nd + 255) / 256;
    long long a0 = 0, a1 = 0, a2 = 0, a3 = 0;
    double q = 0.0;
    for (int i = tid * per; i < nd && i < (tid + 1) * per; i++) {
        const DomPart dp = P.dpart[C.dom_off + i];
        a0 += dp.nv; a1 += dp.nkink; a2 += dp.nw; a3 += dp.occ2; q += dp.qimp;
    }
    // block sum: a butterfly inside each wavefront, then the four wavefront
    // sums (the integer counts are exact in any order; the estimator sum has
    // this fixed order for every launch form)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        a0 += __shfl_xor(a0, o, 64);
        a1 += __shfl_xor(a1, o, 64);
        a2 += __shfl_xor(a2, o, 64);
        a3 += __shfl_xor(a3, o, 64);
        q += __shfl_xor(q, o, 64);
    }
    __shared__ long long s0[4], s1[4], s2[4], s3[4];
    __shared__ double sq[4];
    if ((tid & 63) == 0) {
        const int wv = tid >> 6;
        s0[wv] = a0; s1[wv] = a1; s2[wv] = a2; s3[wv] = a3; sq[wv] = q;
    }
    __syncthreads();
    if (tid == 0) {
        pmwa_obs o;
        o.nv = (s0[0] + s0[1]) + (s0[2] + s0[3]);
        o.nkink = (s1[0] + s1[1]) + (s1[2] + s1[3]);
        o.nw = (s2[0] + s2[1]) + (s2[2] + s2[3]);
        o.occ2 = (s3[0] + s3[1]) + (s3[2] + s3[3]);
        o.qimp = (sq[0] + sq[1]) + (sq[2] + sq[3]);
        o.nn2 = (long long)P.nnacc[chain];
        P.nnacc[chain] = 0ULL;
        const unsigned long long sw = P.sweep[chain];
        P.ser[C.ser_off + (long long)(sw % (unsigned long long)P.series_cap)] = o;
        P.sweep[chain] = sw + 1ULL;
        // running sums and sums of squares, in sweep order
        pmwa_obs_acc a = P.acc[chain];
        a.sweeps += 1;
        a.nv += o.nv; a.nkink += o.nkink; a.nw += o.nw; a.occ2 += o.occ2; a.nn2 += o.nn2;
        a.qimp = a.qimp + o.qimp;
        a.nv_sq = a.nv_sq + (double)o.nv * (double)o.nv;
        a.nkink_sq = a.nkink_sq + (double)o.nkink * (double)o.nkink;
        a.nw_sq = a.nw_sq + (double)o.nw * (double)o.nw;
        a.occ2_sq = a.occ2_sq + (double)o.occ2 * (double)o.occ2;
        a.nn2_sq = a.nn2_sq + (double)o.nn2 * (double)o.nn2;
        a.qimp_sq = a.qimp_sq + o.qimp * o.qimp;
        P.acc[chain] = a;
    }
}

// Restart the accumulated observables of chains [0, n).
__global__ void __launch_bounds__(64) k_reset_acc(Pools P, int n)
{
    for (int c = (int)(blockIdx.x * 64 + threadIdx.x); c < n; c += (int)(gridDim.x * 64)) {
        pmwa_obs_acc z;
        z.sweeps = 0; z.nv = 0; z.nkink = 0; z.nw = 0; z.occ2 = 0; z.nn2 = 0;
        z.qimp = 0.0; z.nv_sq = 0.0; z.nkink_sq = 0.0; z.nw_sq = 0.0; z.occ2_sq = 0.0;
        z.nn2_sq = 0.0; z.qimp_sq = 0.0;
        P.acc[c] = z;
    }
}

// State hash of one chain: one lane per (slab, site), the terms of its
// boundary state, count and events (each site's events are adjacent rows of
// its domain block), summed modulo 2^64 over a wavefront and added to *out.
__global__ void __launch_bounds__(64) k_hash(Pools P, int chain, unsigned long long* __restrict__ out)
{
    const ChainDev& C = P.cd[chain];
    const long long nunits = (long long)C.ntau * C.N;
    const long long u = (long long)blockIdx.x * 64 + threadIdx.x;
    unsigned long long acc = 0ULL;
    if (u < nunits) {
        const int per = C.ndsp * C.nloc;
        const int k = (int)(u / per), rem = (int)(u - (long long)k * per);
        const int dsp = rem / C.nloc, sl = rem - dsp * C.nloc;
        const int site = site_join(C, dsp, sl);
        const uint64_t uc = (uint64_t)k * (uint64_t)C.N + (uint64_t)site;
        const long long su = unit_su(C, k, dsp, sl);
        const int n = P.cnt[C.cnt_off + su];
        const uint32_t b = P.bs[C.bs_off + su];
        acc = mix64((uc << 20) ^ ((uint64_t)n << 1) ^ (uint64_t)b);
        const uint2* E = P.ev + ev_base(C, k, dsp, sl);
        for (int j = 0; j < n; j++) {
            const uint2 e = E[(long long)j * C.nloc];
            acc += mix64(mix64((uc << 15) | (uint64_t)j) ^ (((uint64_t)e.x << 4) | (uint64_t)e.y));
        }
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
    if (threadIdx.x == 0) atomicAdd(out, acc);
}

}  // namespace pmwa
