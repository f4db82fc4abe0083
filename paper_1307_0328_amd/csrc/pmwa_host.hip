// pmwa_host.hip -- C ABI of the gfx950 PMWA sweep (see include/pmwa.h).
//
// Host tables follow the paper's definitions with a fixed floating-point
// operation order (no contraction), so that every Monte Carlo decision is
// reproducible bit for bit by any implementation that uses the same order:
//   Delta = beta / M, lambda = eta * Delta, F[g][v] = expm1(lambda * v * 2^(8g));
//   E_b(sa,sc) = V*(sa&sc) - (mu*0.25)*(sa+sc); C = max E_b + t/2 (t > 0) or
//   + 1/2; w_d = C - E_b; acc = w_d / rho_max;
//   Poisson candidate counts per slab (inversion table, tail folded into a
//   final 2.0 entry); directed-loop pair weights w_ij = w_ji with row sums
//   w_i (minimal bounce), cumulative exit probabilities w_ji / w_i.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

#include "pmwa_device.h"

namespace pmwa {
__global__ void k_vertex(Pools P, const int2* __restrict__ blk, int vs, int cr, int rows, int vmode);
__global__ void k_assemble_w(Pools P, const int2* __restrict__ blk, int nmax);
__global__ void k_assemble(Pools P, const int2* __restrict__ blk);
template <bool HBM_ONLY>
__global__ void k_scatter(Pools P, const int2* __restrict__ blk);
template <int LANES>
__global__ void k_btemporal(Pools P, const int2* __restrict__ blk);
__global__ void k_green(Pools P, int chain, const int4* __restrict__ disp, int nd, int nchunk,
                        double* __restrict__ part);
__global__ void k_bspatial(Pools P, const int2* __restrict__ blk, int d);
__global__ void k_finish(Pools P, const int* __restrict__ chains);
__global__ void k_reset_acc(Pools P, int n);
__global__ void k_hash(Pools P, int chain, unsigned long long* out);
__global__ void k_green_sum(const double* part, int ntau, int nd, int nchunk, double norm, double* out);
__global__ void k_corr(Pools P, int chain, const int4* pts, int npt, int nbase, int nchunk, double* part);
}  // namespace pmwa

using namespace pmwa;

// ---------------------------------------------------------------------------
// Static device scratch of pmwa_green_static, the entry point that allocates
// nothing: the displacements, the per-displacement results and the per-block
// partials of the Green-function kernels.  Each GPU holds its own copy for
// the life of the process; host code reaches it only through the address
// hipGetSymbolAddress returns on that device (kept per device below).
// ---------------------------------------------------------------------------
namespace {
constexpr size_t SCR_DISP = 0;                              // int4[PMWA_GREEN_MAX]
constexpr size_t SCR_OUT = 1024;                            // double[PMWA_GREEN_MAX]
constexpr size_t SCR_PART = 2048;                           // double[PMWA_GREEN_STATIC_PARTIALS]
constexpr size_t SCR_BYTES = SCR_PART + (size_t)PMWA_GREEN_STATIC_PARTIALS * sizeof(double);
static_assert(SCR_OUT >= PMWA_GREEN_MAX * sizeof(int4) && SCR_PART - SCR_OUT >= PMWA_GREEN_MAX * sizeof(double),
              "scratch regions overlap");
constexpr int SCR_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[SCR_MAX_DEVICES] = {};
}  // namespace

static __device__ __align__(256) unsigned char scratch[SCR_BYTES];

// Device address of `scratch` on device `dev` (which must be current),
// looked up once per device.
static int scratch_address(int dev, void** out)
{
    *out = nullptr;
    if (dev < 0 || dev >= SCR_MAX_DEVICES) return PMWA_EDEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || ptr == nullptr) return PMWA_EDEVICE;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return PMWA_OK;
}

namespace {

constexpr int KMAX_TABLE = 1024;   // length bound of the Poisson table construction

struct HostChain {
    pmwa_params p;
    ChainDev d;
    std::vector<double> cdf;        // ntau * cdf_stride
    double C, rho_max, delta;
    int64_t n_units_v, n_units_r, n_dom, n_bt, n_bsx, n_bsy;
    uint64_t enq_sweeps = 0, read_sweeps = 0;
    std::vector<pmwa_obs> host_rows;   // drained, not yet returned
    // what the chain's regions hold (a slot keeps these for every chain it takes)
    int64_t cap_ev = 0, cap_su = 0, cap_bv = 0, cap_dom = 0, cap_cdf = 0, cap_scr = 0, cap_oc = 0;
    int64_t cap_units_v = 0, cap_units_r = 0, cap_bt = 0, cap_bsx = 0, cap_bsy = 0;
    int cap_event = 0;
    bool active = true;
    uint64_t target = ~0ULL;
    // slot installs: pinned staging and the event of its last copy
    unsigned char* staging = nullptr;
    hipEvent_t staged = nullptr;
};

template <typename T>
T* dalloc(size_t n, int* rc)
{
    if (n == 0) n = 1;
    void* p = nullptr;
    if (hipMalloc(&p, n * sizeof(T)) != hipSuccess) { *rc = PMWA_ENOMEM; return nullptr; }
    return static_cast<T*>(p);
}

}  // namespace

// The block tables of one group of chains and the stream it runs on.
struct LaunchGroup {
    std::vector<int> chains;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    hipEvent_t done = nullptr;
    int2 *v = nullptr, *r = nullptr, *s = nullptr, *bt = nullptr, *bsx = nullptr, *bsy = nullptr, *rw = nullptr;
    int nv = 0, nr = 0, ns = 0, nbt = 0, nbsx = 0, nbsy = 0, nrw = 0;
    int* fin = nullptr;        // chain indices of k_finish
    int nfin = 0;
};

struct pmwa_handle {
    hipStream_t stream = nullptr;
    pmwa_opts opts{};
    std::vector<HostChain> ch;
    Pools P{};
    ChainDev* d_cd = nullptr;
    double* d_cdf = nullptr;
    // launch groups: each holds the block tables of its chains and a stream
    // (the first group uses the handle's stream); with more than one group a
    // sweep forks to the group streams and joins back, so a group's phases
    // never wait for another group's
    std::vector<LaunchGroup> grp;
    hipEvent_t fork_ev = nullptr;
    bool regen_wave = false;   // worm re-generation with one wavefront per (site, slab)
    int rw_nmax = 4;           // bond-buffer entries of a site in a slab, at most
    size_t rw_lds = 0;
    size_t lds_bytes = 0;
    bool scatter_hbm = false;   // the scattering kernel's HBM form (nodes, counts in device memory)
    size_t bs_lds = 0;       // LDS of the spatial-boundary kernel
    int bt_lanes = 64;       // lanes per workgroup of the temporal-boundary update (64 or 16)
    int vs = 1;              // candidate column length of the vertex kernel
    int v_rows = 1;          // flips per site staged in LDS by the vertex kernel
    int v_cr = 1;            // candidate rows per lane of the vertex kernel's LDS
    size_t v_lds = 0;
    int64_t ev_total = 0, site_slabs = 0;
    bool slots = false;
    int max_nloc = 1;
    int max_capb = 1;        // the largest bond-buffer capacity (spatial-update LDS)
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    bool own_stream = false;
    // phase timing: events around the phases whose bit (phase - 1) is set
    bool timing = false;
    uint32_t timing_mask = 0;
    std::vector<hipEvent_t> ev_pool;
    std::vector<int> ev_phase;          // phase of the pair (2i, 2i+1)
    size_t ev_used = 0;
    // Green-function measurement: displacements and per-block partials
    int4* d_gdisp = nullptr;
    double* d_gpart = nullptr;
    size_t gpart_cap = 0;
    unsigned long long* d_hash = nullptr;   // result of the state-hash reduction
    int4* d_cpts = nullptr;                 // correlator points
    void* scratch = nullptr;                // this device's static scratch (pmwa_green_static)
};

// ---------------------------------------------------------------------------
// tables
// ---------------------------------------------------------------------------
static double vertex_weight(const double wd[4], double t, int S)
{
    if ((S & 3) == (S >> 2)) return wd[S & 3];
    if (S == 9 || S == 6) return t;
    return 0.0;
}

// w_ij = w_ji, sum_j w_ij = w_i over the allowed exits, fewest bounces
static void pair_weights(const double w[4], double W[4][4])
{
    std::memset(W, 0, sizeof(double) * 16);
    int idx[4], n = 0;
    for (int j = 0; j < 4; j++)
        if (w[j] > 0.0) idx[n++] = j;
    for (int a = 1; a < n; a++) {   // stable, descending weight
        int v = idx[a], b = a - 1;
        while (b >= 0 && w[idx[b]] < w[v]) { idx[b + 1] = idx[b]; b--; }
        idx[b + 1] = v;
    }
    if (n == 0) return;
    if (n == 1) { W[idx[0]][idx[0]] = w[idx[0]]; return; }
    const int ja = idx[0], jb = idx[1], jc = n == 3 ? idx[2] : -1;
    const double a = w[ja], b = w[jb], c = n == 3 ? w[jc] : 0.0;
    if (a <= b + c) {
        W[ja][jb] = W[jb][ja] = ((a + b) - c) * 0.5;
        if (jc >= 0) {
            W[ja][jc] = W[jc][ja] = ((a + c) - b) * 0.5;
            W[jb][jc] = W[jc][jb] = ((b + c) - a) * 0.5;
        }
    } else {
        W[ja][ja] = (a - b) - c;
        W[ja][jb] = W[jb][ja] = b;
        if (jc >= 0) W[ja][jc] = W[jc][ja] = c;
    }
}

static int validate(const pmwa_params& p)
{
    if (p.Lx < 3 || p.Ly < 3) return 0;
    if (!(p.beta > 0.0) || !(p.eta > 0.0) || !(p.t >= 0.0)) return 0;
    if (!std::isfinite(p.V) || !std::isfinite(p.mu) || !std::isfinite(p.beta) || !std::isfinite(p.t)) return 0;
    if (p.dom_x < 1 || p.dom_y < 1 || p.dom_tau < 1 || p.dom_tau > NT_MAX) return 0;
    if (p.Lx % p.dom_x || p.Ly % p.dom_y) return 0;
    if (p.Lx / p.dom_x < 2 || p.Ly / p.dom_y < 2) return 0;
    if (p.ticks_log2 < 8 || p.ticks_log2 > 29) return 0;
    if ((int64_t(1) << p.ticks_log2) / p.dom_tau < 2) return 0;
    if (p.chain_id >= (1u << 24)) return 0;
    if ((int64_t)p.Lx * p.Ly >= (int64_t(1) << 28)) return 0;
    if (p.eta * p.beta > 8.0) return 0;     // worms per interval fit the sampler
    return 1;
}

// mean events per (site, slab): four bonds, each with at most rho_max
// diagonal vertices per unit time plus kinks (~ t), and worms
static double mean_events(const pmwa_params& p, double rho_max)
{
    const double dbeta = p.beta / p.dom_tau;
    return 4.0 * (rho_max + p.t) * dbeta + 2.0 * p.eta * dbeta + 1.0;
}

extern "C" int pmwa_default_event_cap(const pmwa_params* p)
{
    if (!p || !validate(*p)) return PMWA_EINVAL;
    double Eb[4], Emax = 0.0;
    for (int s = 0; s < 4; s++) {
        const int sa = s & 1, sc = s >> 1;
        Eb[s] = p->V * (double)(sa & sc) - (p->mu * 0.25) * (double)(sa + sc);
        if (s == 0 || Eb[s] > Emax) Emax = Eb[s];
    }
    const double C = std::isnan(p->C) ? Emax + (p->t > 0.0 ? 0.5 * p->t : 0.5) : p->C;
    double rho = 0.0;
    for (int s = 0; s < 4; s++) rho = (s == 0 || C - Eb[s] > rho) ? C - Eb[s] : rho;
    const double m = mean_events(*p, rho);
    int cap = (int)std::ceil(m + 10.0 * std::sqrt(m) + 32.0);
    return (cap + 7) & ~7;
}

static int build_chain(const pmwa_params& p, uint32_t cap_override, HostChain& hc)
{
    if (!validate(p)) return PMWA_EINVAL;
    hc.p = p;
    ChainDev& d = hc.d;
    std::memset(&d, 0, sizeof(d));
    d.Lx = p.Lx; d.Ly = p.Ly; d.N = p.Lx * p.Ly; d.ntau = p.dom_tau;
    d.ex = p.Lx / p.dom_x; d.ey = p.Ly / p.dom_y; d.nloc = d.ex * d.ey;
    d.dom_x = p.dom_x; d.dom_y = p.dom_y; d.ndsp = p.dom_x * p.dom_y;
    d.M = 1 << p.ticks_log2;
    d.chain_id = p.chain_id;
    d.key0 = (uint32_t)p.seed; d.key1 = (uint32_t)(p.seed >> 32);
    hc.delta = p.beta / (double)d.M;
    d.lambda = p.eta * hc.delta;
    d.t = p.t;
    for (int g = 0; g < 4; g++)
        for (int v = 0; v < 256; v++)
            d.F[g * 256 + v] = std::expm1(d.lambda * (double)((uint64_t)v << (8 * g)));

    double Eb[4], Emax = 0.0;
    for (int s = 0; s < 4; s++) {
        const int sa = s & 1, sc = s >> 1;
        Eb[s] = p.V * (double)(sa & sc) - (p.mu * 0.25) * (double)(sa + sc);
        if (s == 0 || Eb[s] > Emax) Emax = Eb[s];
    }
    hc.C = std::isnan(p.C) ? Emax + (p.t > 0.0 ? 0.5 * p.t : 0.5) : p.C;
    double wd[4];
    hc.rho_max = 0.0;
    for (int s = 0; s < 4; s++) {
        wd[s] = hc.C - Eb[s];
        if (!(wd[s] > 0.0)) return PMWA_EINVAL;
        if (s == 0 || wd[s] > hc.rho_max) hc.rho_max = wd[s];
    }
    for (int s = 0; s < 4; s++) d.acc[s] = wd[s] / hc.rho_max;
    for (int S = 0; S < 16; S++) d.vw[S] = vertex_weight(wd, p.t, S);
    for (int k = 0; k <= d.ntau; k++) d.T[k] = (int32_t)(((int64_t)k * (int64_t)d.M) / d.ntau);

    // Poisson(rho_max * Delta * dT_k) CDF of candidate counts
    std::vector<std::vector<double>> tabs(d.ntau);
    int stride = 0;
    for (int k = 0; k < d.ntau; k++) {
        const double mu = hc.rho_max * (hc.delta * (double)(d.T[k + 1] - d.T[k]));
        if (!(mu < 500.0)) return PMWA_EINVAL;
        std::vector<double>& t = tabs[k];
        double pj = std::exp(-mu), cum = pj;
        t.push_back(cum);
        int j = 0;
        for (;;) {
            j++;
            pj = (pj * mu) / (double)j;
            if ((double)j > mu && pj < 0x1.0p-64) break;
            if (j >= KMAX_TABLE - 1) break;
            cum = cum + pj;
            t.push_back(cum);
        }
        t.push_back(2.0);
        if ((int)t.size() > KMAXC) return PMWA_EINVAL;
        stride = std::max(stride, (int)t.size());
    }
    d.cdf_stride = stride;
    // bond buffer: candidates plus the kinks kept; the mean number of kinks of
    // a bond in a slab is at most t times the slab's beta
    {
        const double tb = p.t * p.beta / (double)d.ntau;
        d.capb = stride + 16 + (int)std::ceil(2.0 * tb + 6.0 * std::sqrt(tb + 1.0));
    }
    hc.cdf.assign((size_t)d.ntau * stride, 2.0);
    for (int k = 0; k < d.ntau; k++)
        std::copy(tabs[k].begin(), tabs[k].end(), hc.cdf.begin() + (size_t)k * stride);

    // scattering exits
    for (int S0 = 0; S0 < 16; S0++) {
        double w[4];
        for (int j = 0; j < 4; j++) w[j] = vertex_weight(wd, p.t, S0 ^ (1 << j));
        double W[4][4];
        pair_weights(w, W);
        for (int i = 0; i < 4; i++) {
            double* row = &d.scat[S0 * 16 + i * 4];
            if (!(w[i] > 0.0)) { for (int j = 0; j < 4; j++) row[j] = 2.0; continue; }
            int jlast = 0;
            for (int j = 0; j < 4; j++) if (W[j][i] > 0.0) jlast = j;
            double cum = 0.0;
            for (int j = 0; j < 4; j++) {
                cum = cum + W[j][i] / w[i];
                row[j] = (j >= jlast) ? 2.0 : cum;
            }
        }
    }
    const long long nc = p.n_cycle > 0 ? p.n_cycle : (long long)std::ceil(4.0 * hc.C / p.eta);
    if (nc < 1 || nc > 10000000) return PMWA_EINVAL;
    d.ncycle = (int32_t)nc;

    d.cap = cap_override ? (int)cap_override : pmwa_default_event_cap(&p);
    if (d.cap < 1 || d.cap > 32767) return PMWA_EINVAL;   // interval index < 2^15 (stream words)
    if (d.cap < 4 || (int64_t)d.nloc * (d.cap + 2) >= (int64_t)0x7FFFFFFF) return PMWA_EINVAL;
    hc.n_units_v = 2LL * d.ntau * d.N;
    hc.n_units_r = (int64_t)d.ntau * d.N;
    hc.n_dom = (int64_t)d.ntau * d.ndsp;
    d.n_dom = (uint32_t)hc.n_dom;
    hc.n_bt = d.N;
    // spatial boundary units: (cross bond, slab)
    hc.n_bsx = p.dom_x > 1 ? (int64_t)p.Ly * p.dom_x * p.dom_tau : 0;
    hc.n_bsy = p.dom_y > 1 ? (int64_t)p.Lx * p.dom_y * p.dom_tau : 0;
    return PMWA_OK;
}

static void block_table(const std::vector<HostChain>& ch, const std::vector<int>& chains, int per_block,
                        int64_t HostChain::*units, std::vector<int2>& out)
{
    out.clear();
    for (int c : chains) {
        const int64_t n = ch[c].*units;
        for (int64_t b = 0; b < n; b += per_block) out.push_back(make_int2(c, (int)b));
    }
}

// Cross bonds of direction d (0: x, 1: y) for the spatial-boundary kernel, one
// block each.  The bonds along one domain edge in one slab are adjacent in
// the table (x-crossing bonds along y, y-crossing bonds along x), and runs of
// 16 entries go to one XCD (workgroups are dealt round-robin over the 8
// XCDs), so that blocks reading the same cache lines of the site-interleaved
// event arrays share an L2.  The units are independent, so the order changes
// no result.  Entries past the end carry an out-of-range unit: their block
// returns at once.
static void spatial_table(const std::vector<HostChain>& ch, const std::vector<int>& chains, int d,
                          std::vector<int2>& out)
{
    std::vector<int2> items;
    for (int c : chains) {
        const HostChain& hc = ch[c];
        const int64_t n = d == 0 ? hc.n_bsx : hc.n_bsy;
        if (n <= 0) continue;
        const int nt = hc.p.dom_tau;
        const int outer = d == 0 ? hc.p.dom_x : hc.p.dom_y;   // the domain column (row)
        const int inner = d == 0 ? hc.p.Ly : hc.p.Lx;         // position along the edge
        for (int o = 0; o < outer; o++)
            for (int k = 0; k < nt; k++)
                for (int i = 0; i < inner; i++) {
                    const int64_t u = d == 0 ? (int64_t)i * hc.p.dom_x + o : (int64_t)o * hc.p.Lx + i;
                    items.push_back(make_int2(c, (int)(u * nt + k)));
                }
    }
    out.clear();
    if (items.empty()) return;
    constexpr int64_t XCD = 8, RUN = 16;
    const int64_t n = (int64_t)items.size();
    const int64_t nb = (n + XCD * RUN - 1) / (XCD * RUN) * (XCD * RUN);
    out.assign((size_t)nb, make_int2(items[0].x, 0x7FFFFFFF));
    for (int64_t b = 0; b < nb; b++) {
        const int64_t x = b % XCD, i = b / XCD;
        const int64_t item = ((i / RUN) * XCD + x) * RUN + (i % RUN);
        if (item < n) out[(size_t)b] = items[(size_t)item];
    }
}

// expected work of one scattering domain of a chain: its expected nodes
// (4 (rho_max + t) beta per site and slab, the vertex ends) and attempts
// (N_cycle times the worms, ~ 4 C beta per site and slab)
static double domain_work(const HostChain& hc)
{
    const double db = hc.p.beta / hc.p.dom_tau;
    return (double)hc.d.nloc * db * (4.0 * (hc.rho_max + hc.p.t) + 4.0 * hc.C);
}

#define HIPCHK(x)                                  \
    do {                                           \
        if ((x) != hipSuccess) return PMWA_EDEVICE; \
    } while (0)

// Allow `bytes` of dynamic LDS for kernel `f`: PMWA_EINVAL beyond the CU's
// LDS, PMWA_EDEVICE if the runtime refuses.
static int set_lds(const void* f, size_t bytes, size_t lds_max)
{
    if (bytes > lds_max) return PMWA_EINVAL;
    if (bytes > 64 * 1024 &&
        hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes) != hipSuccess)
        return PMWA_EDEVICE;
    return PMWA_OK;
}

static int upload_table(const std::vector<int2>& t, int2** dst, int* n)
{
    *n = (int)t.size();
    if (t.empty()) { *dst = nullptr; return PMWA_OK; }
    if (hipMalloc(dst, t.size() * sizeof(int2)) != hipSuccess) return PMWA_ENOMEM;
    HIPCHK(hipMemcpy(*dst, t.data(), t.size() * sizeof(int2), hipMemcpyHostToDevice));
    return PMWA_OK;
}

// ---------------------------------------------------------------------------
// launches
// ---------------------------------------------------------------------------
static int launch_kernel(pmwa_t* h, int phase, const LaunchGroup& g);

static int launch_phase(pmwa_t* h, int phase, const LaunchGroup& g)
{
    if (!h->timing || !((h->timing_mask >> (phase - 1)) & 1u)) return launch_kernel(h, phase, g);
    if (h->ev_used + 2 > h->ev_pool.size()) {
        for (int i = 0; i < 2; i++) {
            hipEvent_t e;
            HIPCHK(hipEventCreate(&e));
            h->ev_pool.push_back(e);
        }
    }
    hipEvent_t e0 = h->ev_pool[h->ev_used], e1 = h->ev_pool[h->ev_used + 1];
    HIPCHK(hipEventRecord(e0, g.stream));
    int rc = launch_kernel(h, phase, g);
    HIPCHK(hipEventRecord(e1, g.stream));
    if (h->ev_phase.size() < h->ev_used / 2 + 1) h->ev_phase.resize(h->ev_used / 2 + 1);
    h->ev_phase[h->ev_used / 2] = phase;
    h->ev_used += 2;
    return rc;
}

static int launch_kernel(pmwa_t* h, int phase, const LaunchGroup& g)
{
    hipStream_t s = g.stream;
    switch (phase) {
    case 1:
        if (g.nv) hipLaunchKernelGGL(k_vertex, dim3(g.nv), dim3(VL), h->v_lds, s, h->P, g.v, h->vs, h->v_cr,
                                     h->v_rows, h->opts.vertex_mode);
        break;
    case 2:
        if (h->regen_wave) {
            if (g.nrw) hipLaunchKernelGGL(k_assemble_w, dim3(g.nrw), dim3(64), h->rw_lds, s, h->P, g.rw, h->rw_nmax);
        } else if (g.nr) {
            hipLaunchKernelGGL(k_assemble, dim3(g.nr), dim3(64), 0, s, h->P, g.r);
        }
        break;
    case 3:
        if (g.ns) {
            if (h->scatter_hbm)
                hipLaunchKernelGGL(k_scatter<true>, dim3(g.ns), dim3(64), h->lds_bytes, s, h->P, g.s);
            else
                hipLaunchKernelGGL(k_scatter<false>, dim3(g.ns), dim3(64), h->lds_bytes, s, h->P, g.s);
        }
        break;
    case 4:
        if (g.nbt) {
            if (h->bt_lanes == 16)
                hipLaunchKernelGGL(k_btemporal<16>, dim3(g.nbt), dim3(16), 0, s, h->P, g.bt);
            else
                hipLaunchKernelGGL(k_btemporal<64>, dim3(g.nbt), dim3(64), 0, s, h->P, g.bt);
        }
        break;
    case 5:
        if (g.nbsx) hipLaunchKernelGGL(k_bspatial, dim3(g.nbsx), dim3(64), h->bs_lds, s, h->P, g.bsx, 0);
        break;
    case 6:
        if (g.nbsy) hipLaunchKernelGGL(k_bspatial, dim3(g.nbsy), dim3(64), h->bs_lds, s, h->P, g.bsy, 1);
        break;
    case 7:
        if (g.nfin) hipLaunchKernelGGL(k_finish, dim3((unsigned)g.nfin), dim3(256), 0, s, h->P, g.fin);
        break;
    default:
        return PMWA_EINVAL;
    }
    return hipGetLastError() == hipSuccess ? PMWA_OK : PMWA_EDEVICE;
}

// Phases [p0, p1] of every group: with one group on the handle's stream;
// with several, forked from the handle's stream to the group streams and
// joined back, so each group advances on its own.
static int launch_phases(pmwa_t* h, int p0, int p1)
{
    if (h->grp.size() == 1) {
        for (int ph = p0; ph <= p1; ph++) {
            int rc = launch_phase(h, ph, h->grp[0]);
            if (rc) return rc;
        }
        return PMWA_OK;
    }
    HIPCHK(hipEventRecord(h->fork_ev, h->stream));
    for (auto& g : h->grp) {
        if (g.stream != h->stream) HIPCHK(hipStreamWaitEvent(g.stream, h->fork_ev, 0));
        for (int ph = p0; ph <= p1; ph++) {
            int rc = launch_phase(h, ph, g);
            if (rc) return rc;
        }
        if (g.stream != h->stream) HIPCHK(hipEventRecord(g.done, g.stream));
    }
    for (auto& g : h->grp)
        if (g.stream != h->stream) HIPCHK(hipStreamWaitEvent(h->stream, g.done, 0));
    return PMWA_OK;
}

static int drain(pmwa_t* h)
{
    HIPCHK(hipStreamSynchronize(h->stream));
    const int cap = h->opts.series_cap;
    for (size_t c = 0; c < h->ch.size(); c++) {
        HostChain& hc = h->ch[c];
        while (hc.read_sweeps < hc.enq_sweeps) {
            const uint64_t slot = hc.read_sweeps % (uint64_t)cap;
            const uint64_t n = std::min<uint64_t>(hc.enq_sweeps - hc.read_sweeps, (uint64_t)cap - slot);
            const size_t o = hc.host_rows.size();
            hc.host_rows.resize(o + n);
            HIPCHK(hipMemcpy(hc.host_rows.data() + o, h->P.ser + hc.d.ser_off + slot,
                             n * sizeof(pmwa_obs), hipMemcpyDeviceToHost));
            hc.read_sweeps += n;
        }
    }
    return PMWA_OK;
}

static int read_flags(pmwa_t* h, std::vector<unsigned int>& f)
{
    HIPCHK(hipStreamSynchronize(h->stream));
    f.resize(h->ch.size());
    HIPCHK(hipMemcpy(f.data(), h->P.flags, f.size() * sizeof(unsigned int), hipMemcpyDeviceToHost));
    return PMWA_OK;
}

static int flag_code(unsigned int f)
{
    if (f & FL_OVERFLOW) return PMWA_EOVERFLOW;
    if (f) return PMWA_ESTATE;
    return PMWA_OK;
}

extern "C" {

const char* pmwa_strerror(int code)
{
    switch (code) {
    case PMWA_OK: return "ok";
    case PMWA_EINVAL: return "invalid argument";
    case PMWA_ENOMEM: return "out of memory";
    case PMWA_EDEVICE: return "HIP error";
    case PMWA_EOVERFLOW: return "capacity overflow (chain state invalid)";
    case PMWA_ESTATE: return "inconsistent state";
    default: return "unknown error";
    }
}

void pmwa_destroy(pmwa_t* h)
{
    if (!h) return;
    (void)hipStreamSynchronize(h->stream);
    if (h->gexec) (void)hipGraphExecDestroy(h->gexec);
    if (h->graph) (void)hipGraphDestroy(h->graph);
    for (hipEvent_t e : h->ev_pool) (void)hipEventDestroy(e);
    for (auto& hc : h->ch) {
        if (hc.staging) (void)hipHostFree(hc.staging);
        if (hc.staged) (void)hipEventDestroy(hc.staged);
    }
    for (auto& g : h->grp) {
        void* gp[] = {g.v, g.r, g.s, g.bt, g.bsx, g.bsy, g.rw, g.fin};
        for (void* p : gp)
            if (p) (void)hipFree(p);
        if (g.done) (void)hipEventDestroy(g.done);
        if (g.own_stream) (void)hipStreamDestroy(g.stream);
    }
    if (h->fork_ev) (void)hipEventDestroy(h->fork_ev);
    if (h->own_stream) (void)hipStreamDestroy(h->stream);
    void* ptrs[] = {h->d_cd, h->d_cdf, h->P.ev, h->P.cnt, h->P.bs, h->P.bv, h->P.bvc, h->P.dpart,
                    h->P.ser, h->P.sweep, h->P.flags, h->P.nnacc, h->P.s_nd, h->P.s_wl, h->P.s_own, h->P.s_oc, h->d_gdisp, h->d_gpart,
                    h->P.acc, h->d_hash, h->d_cpts};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    delete h;
}

static int create_impl(const pmwa_params* chains, int n_chains, const pmwa_opts* opts, bool slots,
                       pmwa_t** out)
{
    if (!out) return PMWA_EINVAL;
    *out = nullptr;
    if (!chains || n_chains < 1 || n_chains > (1 << 20)) return PMWA_EINVAL;
    pmwa_t* h = new (std::nothrow) pmwa_handle();
    if (!h) return PMWA_ENOMEM;
    if (opts) h->opts = *opts;
    if (h->opts.series_cap <= 0) h->opts.series_cap = 4096;
    if (h->opts.scatter_mode < 0 || h->opts.scatter_mode > 2 || h->opts.event_cap < 0 ||
        h->opts.event_cap > 32767 || h->opts.regen_mode < 0 || h->opts.regen_mode > 2 ||
        h->opts.vertex_mode < 0 || h->opts.vertex_mode > 3 || h->opts.scatter_lds < 0 ||
        h->opts.scatter_lds > 160 * 1024 || h->opts.groups < 0 || h->opts.groups > 64 ||
        (h->opts.vertex_rows != 0 && (h->opts.vertex_rows < 8 || h->opts.vertex_rows > 128))) {
        delete h;
        return PMWA_EINVAL;
    }
    h->stream = (hipStream_t)h->opts.stream;
    if (!h->stream) {
        // work goes to a stream of the handle (default priority)
        if (hipStreamCreate(&h->stream) != hipSuccess) { delete h; return PMWA_EDEVICE; }
        h->own_stream = true;
    }
    h->ch.resize(n_chains);
    int rc = PMWA_OK;
    int64_t ev = 0, su = 0, bv = 0, bvc = 0, dom = 0, cdf = 0, scr = 0, oc = 0;
    int max_nloc = 1;
    for (int c = 0; c < n_chains && rc == PMWA_OK; c++) {
        HostChain& hc = h->ch[c];
        rc = build_chain(chains[c], (uint32_t)h->opts.event_cap, hc);
        if (rc) break;
        ChainDev& d = hc.d;
        d.ev_off = ev; ev += (int64_t)d.ntau * d.N * d.cap;
        d.cnt_off = su; d.bs_off = su; su += (int64_t)d.ntau * d.N;
        d.bv_off = bv; bv += 2LL * d.ntau * d.N * d.capb;
        d.bvc_off = bvc; bvc += 2LL * d.ntau * d.N;
        d.dom_off = dom; dom += hc.n_dom;
        d.ser_off = (int64_t)c * h->opts.series_cap;
        d.cdf_off = cdf; cdf += (int64_t)hc.cdf.size();
        max_nloc = std::max(max_nloc, d.nloc);
        hc.cap_ev = (int64_t)d.ntau * d.N * d.cap;
        hc.cap_su = (int64_t)d.ntau * d.N;
        hc.cap_bv = 2LL * d.ntau * d.N * d.capb;
        hc.cap_dom = hc.n_dom;
        hc.cap_cdf = (int64_t)hc.cdf.size();
        hc.cap_units_v = hc.n_units_v; hc.cap_units_r = hc.n_units_r;
        hc.cap_bt = hc.n_bt; hc.cap_bsx = hc.n_bsx; hc.cap_bsy = hc.n_bsy;
        hc.cap_event = d.cap;
        hc.active = !slots;
        hc.target = slots ? 0ULL : ~0ULL;
        d.active = slots ? 0 : 1;
        d.target = slots ? 0 : INT64_MAX;
    }
    if (rc) { pmwa_destroy(h); return rc; }
    h->slots = slots;
    h->max_nloc = max_nloc;

    // LDS budget of the scattering kernel
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        pmwa_destroy(h);
        return PMWA_EDEVICE;
    }
    if (int e = scratch_address(dev, &h->scratch)) {
        pmwa_destroy(h);
        return e;
    }
    size_t lds_max = prop.sharedMemPerBlock;
    if (prop.maxSharedMemoryPerMultiProcessor > lds_max) lds_max = prop.maxSharedMemoryPerMultiProcessor;
    if (lds_max > 160 * 1024) lds_max = 160 * 1024;
    // LDS form of the scattering kernel: the exit thresholds, the stream ring,
    // the per-site offsets and counts, then 12 bytes per node (and the worm
    // list).  Sized for the largest expected domain within the CU's LDS;
    // larger domains take the HBM store.  opts.scatter_lds (bytes) overrides.
    const size_t fixed = 768 * sizeof(uint64_t) + (size_t)(2 * max_nloc + 1) * sizeof(int);
    const size_t fixed_al = (fixed + 15) & ~(size_t)15;
    double want = 0.0;                 // nodes of the largest expected domain, with margin
    for (auto& hc : h->ch) {
        const double m = mean_events(hc.p, hc.rho_max) * 0.75;
        want = std::max(want, hc.d.nloc * (m * 1.3 + 2.0) + 64.0);
    }
    const int smode = h->opts.scatter_mode;
    size_t lds = 0;
    if (smode != 2) {
        lds = h->opts.scatter_lds > 0 ? (size_t)h->opts.scatter_lds
                                      : fixed_al + (size_t)std::ceil(want * 12.5) + 256;
        // many domains: at most 80 KB, so that two domains share a CU (the
        // larger ones take the HBM store); measured best on the 256-chain batch
        int64_t ndom = 0;
        for (auto& hc : h->ch) ndom += hc.n_dom;
        if (h->opts.scatter_lds == 0 && ndom >= 2LL * std::max(prop.multiProcessorCount, 1)) {
            lds = std::min<size_t>(lds, 80 * 1024);
            // when no chain's typical domain fits even then, every domain takes
            // the HBM store: a third of the CU's LDS, rounded down to 2 KB so
            // that three domains share a CU whatever the allocation granule,
            // each keeping its owner stamps (one per node pair) in LDS.
            // Measured on 2048^2 with 32x32 sites x beta*t 4 domains (18-20k
            // nodes): 52 KB 30.3 ms; 56-80 KB (two per CU) 35.4; 48 KB with the
            // stamps in HBM 36.4; 16 KB 42.0; the 6 KB HBM form 46.2.
            bool any_fits = false;
            for (auto& hc : h->ch) {
                const double typ = hc.d.nloc * (mean_events(hc.p, hc.rho_max) * 0.5 + 2.0);
                if ((double)fixed_al + 12.0 * typ + 256.0 <= (double)lds) any_fits = true;
            }
            if (!any_fits) lds = std::max<size_t>(fixed_al + 64, (lds_max / 3) & ~(size_t)2047);
        }
        lds = std::min(lds, lds_max);
        lds = std::max(lds, fixed_al + 64);
        lds = (lds + 15) & ~(size_t)15;
        if (lds > lds_max) lds = 0;        // not even the fixed region fits: HBM form
    }
    h->scatter_hbm = lds == 0;
    h->P.lds_bytes = (int32_t)lds;
    h->lds_bytes = h->scatter_hbm ? 768 * sizeof(uint64_t) + 16 : lds;
    {
        const int e = h->scatter_hbm ? set_lds((const void*)k_scatter<true>, h->lds_bytes, lds_max)
                                     : set_lds((const void*)k_scatter<false>, h->lds_bytes, lds_max);
        if (e) {
            pmwa_destroy(h);
            return e;
        }
    }
    // HBM node scratch for domains beyond the LDS capacity
    for (auto& hc : h->ch) {
        ChainDev& d = hc.d;
        const double m = mean_events(hc.p, hc.rho_max);
        int64_t nodes = (int64_t)std::ceil(d.nloc * (m + 4.0 * std::sqrt(m) + 8.0)) + 2 * d.nloc + 64;
        nodes = std::min<int64_t>(nodes, (int64_t)d.nloc * (d.cap + 2));
        nodes = std::min<int64_t>(nodes, (int64_t)PX_NIL - 1);   // partner links are 24-bit
        d.scr_nodes = (int32_t)nodes;
        d.scr_off = scr;
        scr += nodes * hc.n_dom;
        hc.cap_scr = nodes * hc.n_dom;
        d.oc_off = oc;
        hc.cap_oc = hc.n_dom * (2LL * d.nloc + 2);
        oc += hc.cap_oc;
    }

    h->ev_total = ev;
    h->site_slabs = su;
    h->P.ev = dalloc<uint2>(ev, &rc);
    h->P.cnt = dalloc<int32_t>(su, &rc);
    h->P.bs = dalloc<uint8_t>(su, &rc);
    h->P.bv = dalloc<uint32_t>(bv, &rc);
    h->P.bvc = dalloc<int32_t>(bvc, &rc);
    h->P.dpart = dalloc<DomPart>(dom, &rc);
    h->P.ser = dalloc<pmwa_obs>((size_t)n_chains * h->opts.series_cap, &rc);
    h->P.sweep = dalloc<unsigned long long>(n_chains, &rc);
    h->P.flags = dalloc<unsigned int>(n_chains, &rc);
    h->P.nnacc = dalloc<unsigned long long>(n_chains, &rc);
    h->P.acc = dalloc<pmwa_obs_acc>(n_chains, &rc);
    h->d_hash = dalloc<unsigned long long>(1, &rc);
    h->P.s_nd = dalloc<uint4>(scr, &rc);
    h->P.s_wl = dalloc<uint32_t>(scr, &rc);
    h->P.s_own = dalloc<uint32_t>(scr, &rc);
    h->P.s_oc = dalloc<int32_t>(oc, &rc);
    h->d_cd = dalloc<ChainDev>(n_chains, &rc);
    h->d_cdf = dalloc<double>(cdf, &rc);
    if (rc) { pmwa_destroy(h); return rc; }
    h->P.cd = h->d_cd;
    h->P.cdf = h->d_cdf;
    h->P.series_cap = h->opts.series_cap;

    std::vector<ChainDev> cds(n_chains);
    std::vector<double> cdfs(std::max<int64_t>(cdf, 1));
    for (int c = 0; c < n_chains; c++) {
        cds[c] = h->ch[c].d;
        std::copy(h->ch[c].cdf.begin(), h->ch[c].cdf.end(), cdfs.begin() + h->ch[c].d.cdf_off);
    }
    std::vector<int2> t;
    int r2 = PMWA_OK;
    if (hipMemcpy(h->d_cd, cds.data(), n_chains * sizeof(ChainDev), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(h->d_cdf, cdfs.data(), cdf * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
        r2 = PMWA_EDEVICE;
    {
        // the temporal update in 16-lane groups where 64-lane ones would
        // leave CUs idle (fewer units than 64 per CU)
        int64_t units = 0;
        for (auto& hc : h->ch) units += hc.n_bt;
        h->bt_lanes = units < 64LL * std::max(prop.multiProcessorCount, 1) ? 16 : 64;
    }
    {
        // worm re-generation: one lane per (site, slab), or one wavefront
        // where there are too few units for lanes to fill the device
        int64_t units = 0;
        int maxcapb = 1;
        for (auto& hc : h->ch) {
            units += hc.n_units_r;
            maxcapb = std::max(maxcapb, hc.d.capb);
        }
        const int mode = h->opts.regen_mode;
        h->regen_wave = mode == 2 || (mode == 0 && units <= 65536);
        h->rw_nmax = 4 * maxcapb;
        h->rw_lds = (size_t)((h->rw_nmax + 3) & ~3) * sizeof(uint32_t) +
                    (size_t)h->rw_nmax * (2 * sizeof(uint32_t) + 2) + (size_t)RW_POOL * sizeof(int32_t);
        if (h->regen_wave) {
            const int e = set_lds((const void*)k_assemble_w, h->rw_lds, lds_max);
            // the lane form needs no LDS: take it when the wavefront form does not fit
            if (e == PMWA_EINVAL && mode == 0) h->regen_wave = false;
            else if (e && !r2) r2 = e;
        }
    }
    // launch groups: chains split by expected work (largest first, each to
    // the lightest group); within a group the scattering domains of the
    // heaviest chains are dispatched first, so that a launch does not end
    // waiting for a large domain started last
    if (!r2) {
        const int G = slots ? 1 : std::max(1, std::min(h->opts.groups, n_chains));
        std::vector<int> order(n_chains);
        for (int c = 0; c < n_chains; c++) order[c] = c;
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
            return domain_work(h->ch[a]) * h->ch[a].n_dom > domain_work(h->ch[b]) * h->ch[b].n_dom;
        });
        h->grp.resize(G);
        std::vector<double> load(G, 0.0);
        for (int c : order) {
            const int g = (int)(std::min_element(load.begin(), load.end()) - load.begin());
            h->grp[g].chains.push_back(c);
            load[g] += domain_work(h->ch[c]) * h->ch[c].n_dom;
        }
        for (int g = 0; g < G && !r2; g++) {
            LaunchGroup& L = h->grp[g];
            std::sort(L.chains.begin(), L.chains.end());
            if (g == 0) L.stream = h->stream;
            else if (hipStreamCreate(&L.stream) != hipSuccess) { r2 = PMWA_EDEVICE; break; }
            else L.own_stream = true;
            if (G > 1 && hipEventCreateWithFlags(&L.done, hipEventDisableTiming) != hipSuccess) { r2 = PMWA_EDEVICE; break; }
            std::vector<int> heavy = L.chains;
            std::stable_sort(heavy.begin(), heavy.end(),
                             [&](int a, int b) { return domain_work(h->ch[a]) > domain_work(h->ch[b]); });
            block_table(h->ch, L.chains, VL, &HostChain::n_units_v, t); if (!r2) r2 = upload_table(t, &L.v, &L.nv);
            block_table(h->ch, L.chains, 64, &HostChain::n_units_r, t); if (!r2) r2 = upload_table(t, &L.r, &L.nr);
            block_table(h->ch, heavy, 1, &HostChain::n_dom, t); if (!r2) r2 = upload_table(t, &L.s, &L.ns);
            block_table(h->ch, L.chains, h->bt_lanes, &HostChain::n_bt, t); if (!r2) r2 = upload_table(t, &L.bt, &L.nbt);
            spatial_table(h->ch, L.chains, 0, t); if (!r2) r2 = upload_table(t, &L.bsx, &L.nbsx);
            spatial_table(h->ch, L.chains, 1, t); if (!r2) r2 = upload_table(t, &L.bsy, &L.nbsy);
            if (h->regen_wave) {
                block_table(h->ch, L.chains, 1, &HostChain::n_units_r, t);
                if (!r2) r2 = upload_table(t, &L.rw, &L.nrw);
            }
            if (!r2) {
                L.nfin = (int)L.chains.size();
                if (hipMalloc(&L.fin, L.nfin * sizeof(int)) != hipSuccess) r2 = PMWA_ENOMEM;
                else if (hipMemcpy(L.fin, L.chains.data(), L.nfin * sizeof(int), hipMemcpyHostToDevice) != hipSuccess)
                    r2 = PMWA_EDEVICE;
            }
        }
        if (!r2 && G > 1 && hipEventCreateWithFlags(&h->fork_ev, hipEventDisableTiming) != hipSuccess) r2 = PMWA_EDEVICE;
    }
    {
        int maxcap = 0, maxcapb = 0;
        for (auto& hc : h->ch) {
            maxcap = std::max(maxcap, hc.d.cap);
            maxcapb = std::max(maxcapb, hc.d.capb);
        }
        // A, B and eight 16-bit arrays per event; per bond vertex its record
        // and two indices; the worm-offset pool
        h->max_capb = maxcapb;
        h->bs_lds = (size_t)maxcap * (2 * sizeof(uint2) + 8 * sizeof(int16_t)) +
                    (size_t)maxcapb * (sizeof(BsVert) + 2 * sizeof(int)) + (size_t)RW_POOL * sizeof(int32_t) + 16;
        // the spatial update holds a cross bond's two site lists in LDS: a
        // chain with spatial domains needs its event capacity to fit
        bool any_spatial = false;
        for (auto& hc : h->ch) any_spatial |= hc.n_bsx > 0 || hc.n_bsy > 0 || slots;
        if (any_spatial && !r2) r2 = set_lds((const void*)k_bspatial, h->bs_lds, lds_max);
        int vs = 1;
        for (auto& hc : h->ch) vs = std::max(vs, hc.d.cdf_stride);
        h->vs = vs;
        // occupation-changing objects (kinks and worms) of a site in a slab
        // staged in LDS; a lane with more reads its lists from HBM
        // per lane: candidate rows, 32 (what the register sort takes) or more
        // if the table is longer than those and the two flip columns, which
        // a lane with more candidates continues into
        auto cand_rows = [&](int rw) { return std::min(vs, std::max(32, vs - 2 * rw)); };
        auto vlds = [&](int rw) {
            return (size_t)vs * 2 * sizeof(double) + ((size_t)cand_rows(rw) + 2 * (size_t)rw) * VL * sizeof(uint32_t);
        };
        // rows per lane.  When every block of the vertex launch is resident
        // at once with 64 rows, LDS does not limit it: 64 (the 64x64 chain,
        // one block per CU: 32 rows made it 2.5x slower, since a wavefront
        // waits for its lanes that walk their lists in HBM).  Otherwise the
        // expected occupation changes of a (site, slab) plus two standard
        // deviations, in steps of 8.  Kinks dominate: about 0.6 t per bond
        // and unit time in the hard-core model (its kinetic energy per bond),
        // four bonds per site; worms add 2 eta per unit time.  Each row costs
        // 512 bytes of the block's LDS, and fewer rows let more blocks share
        // a CU: measured on the 256-chain batch, 32 rows at slabs of beta*t 8
        // and 24 at 4 are the fastest (64 rows: 16-55% slower; 24 and 16
        // rows: a factor 2 at slabs of 8)
        int rows = h->opts.vertex_rows;
        int64_t vblocks = 0;
        for (auto& hc : h->ch) vblocks += (hc.n_units_v + VL - 1) / VL;
        const size_t lds64 = vlds(64);
        const int64_t resident64 = (int64_t)std::max(prop.multiProcessorCount, 1) *
                                   std::max<int64_t>(1, (int64_t)(lds_max / lds64));
        if (rows == 0 && vblocks <= resident64) rows = std::min(std::max(maxcap, 8), 64);
        if (rows == 0) {
            double f = 0.0;
            for (auto& hc : h->ch) {
                const double db = hc.p.beta / hc.p.dom_tau;
                f = std::max(f, 2.5 * hc.p.t * db + 2.0 * hc.p.eta * db + 1.0);
            }
            rows = ((int)std::ceil(f + 2.0 * std::sqrt(f)) + 7) & ~7;
            rows = std::max(16, std::min(rows, std::min(std::max(maxcap, 8), 64)));
        }
        h->v_rows = rows;
        h->v_cr = cand_rows(rows);
        h->v_lds = vlds(rows);
        if (!r2) r2 = set_lds((const void*)k_vertex, h->v_lds, lds_max);
    }
    if (r2) { pmwa_destroy(h); return r2; }
    // the empty configuration
    if (hipMemsetAsync(h->P.cnt, 0, su * sizeof(int32_t), h->stream) != hipSuccess ||
        hipMemsetAsync(h->P.bs, 0, su, h->stream) != hipSuccess ||
        hipMemsetAsync(h->P.sweep, 0, n_chains * sizeof(unsigned long long), h->stream) != hipSuccess ||
        hipMemsetAsync(h->P.flags, 0, n_chains * sizeof(unsigned int), h->stream) != hipSuccess ||
        hipMemsetAsync(h->P.nnacc, 0, n_chains * sizeof(unsigned long long), h->stream) != hipSuccess ||
        hipMemsetAsync(h->P.acc, 0, n_chains * sizeof(pmwa_obs_acc), h->stream) != hipSuccess ||
        hipMemsetAsync(h->P.bvc, 0, std::max<int64_t>(bvc, 1) * sizeof(int32_t), h->stream) != hipSuccess ||
        hipMemsetAsync(h->P.dpart, 0, std::max<int64_t>(dom, 1) * sizeof(DomPart), h->stream) != hipSuccess ||
        hipStreamSynchronize(h->stream) != hipSuccess) {
        pmwa_destroy(h);
        return PMWA_EDEVICE;
    }
    if (slots) {
        for (auto& hc : h->ch) {
            if (hipHostMalloc((void**)&hc.staging, sizeof(ChainDev) + hc.cap_cdf * sizeof(double)) != hipSuccess ||
                hipEventCreateWithFlags(&hc.staged, hipEventDisableTiming) != hipSuccess) {
                pmwa_destroy(h);
                return PMWA_ENOMEM;
            }
        }
    }
    *out = h;
    return PMWA_OK;
}

int pmwa_create(const pmwa_params* chains, int n_chains, const pmwa_opts* opts, pmwa_t** out)
{
    return create_impl(chains, n_chains, opts, false, out);
}

int pmwa_create_slots(const pmwa_params* shapes, int n_slots, const pmwa_opts* opts, pmwa_t** out)
{
    return create_impl(shapes, n_slots, opts, true, out);
}

static void advance_enq(pmwa_t* h)
{
    for (auto& hc : h->ch)
        if (hc.active && hc.enq_sweeps < hc.target) hc.enq_sweeps++;
}

// Build the chain `p` with the event capacity of slot `slot` and check that it
// fits the slot's regions and launch tables.
static int slot_fit(pmwa_t* h, int slot, const pmwa_params* p, HostChain& job)
{
    const HostChain& hc = h->ch[slot];
    int rc = build_chain(*p, (uint32_t)hc.cap_event, job);
    if (rc) return rc;
    const ChainDev& d = job.d;
    const int64_t ev = (int64_t)d.ntau * d.N * d.cap, su = (int64_t)d.ntau * d.N;
    const int64_t bv = 2LL * d.ntau * d.N * d.capb;
    if (ev > hc.cap_ev || su > hc.cap_su || bv > hc.cap_bv || job.n_dom > hc.cap_dom ||
        (int64_t)job.cdf.size() > hc.cap_cdf || job.n_units_v > hc.cap_units_v ||
        job.n_units_r > hc.cap_units_r || job.n_bt > hc.cap_bt || job.n_bsx > hc.cap_bsx ||
        job.n_bsy > hc.cap_bsy || d.nloc > h->max_nloc || d.cdf_stride > h->vs ||
        (h->regen_wave && 4 * d.capb > h->rw_nmax) || job.n_dom * (2LL * d.nloc + 2) > hc.cap_oc ||
        d.capb > h->max_capb)
        return PMWA_EINVAL;
    return PMWA_OK;
}

int pmwa_slot_fits(pmwa_t* h, int slot, const pmwa_params* p)
{
    if (!h || !p || !h->slots || slot < 0 || slot >= (int)h->ch.size()) return PMWA_EINVAL;
    HostChain job;
    return slot_fit(h, slot, p, job);
}

int pmwa_slot_load(pmwa_t* h, int slot, const pmwa_params* p, int64_t target_sweeps)
{
    if (!h || !p || !h->slots || slot < 0 || slot >= (int)h->ch.size() || target_sweeps < 0) return PMWA_EINVAL;
    HostChain& hc = h->ch[slot];
    HostChain job;
    int rc = slot_fit(h, slot, p, job);
    if (rc) return rc;
    ChainDev& d = job.d;
    const int64_t su = (int64_t)d.ntau * d.N;
    const ChainDev& s = hc.d;
    d.ev_off = s.ev_off; d.cnt_off = s.cnt_off; d.bs_off = s.bs_off; d.bv_off = s.bv_off;
    d.bvc_off = s.bvc_off; d.dom_off = s.dom_off; d.ser_off = s.ser_off; d.cdf_off = s.cdf_off;
    d.scr_off = s.scr_off;
    d.oc_off = s.oc_off;
    d.scr_nodes = (int32_t)std::min<int64_t>(hc.cap_scr / std::max<int64_t>(job.n_dom, 1), 0x7FFFFFFF);
    d.active = 1;
    d.target = target_sweeps;
    // the staging buffer of the slot's previous install must have been consumed
    HIPCHK(hipEventSynchronize(hc.staged));
    std::memcpy(hc.staging, &d, sizeof(ChainDev));
    std::memcpy(hc.staging + sizeof(ChainDev), job.cdf.data(), job.cdf.size() * sizeof(double));
    hipStream_t st = h->stream;
    HIPCHK(hipMemcpyAsync(h->d_cd + slot, hc.staging, sizeof(ChainDev), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(h->d_cdf + d.cdf_off, hc.staging + sizeof(ChainDev), job.cdf.size() * sizeof(double),
                          hipMemcpyHostToDevice, st));
    HIPCHK(hipEventRecord(hc.staged, st));
    // the empty configuration
    HIPCHK(hipMemsetAsync(h->P.cnt + d.cnt_off, 0, su * sizeof(int32_t), st));
    HIPCHK(hipMemsetAsync(h->P.bs + d.bs_off, 0, su, st));
    HIPCHK(hipMemsetAsync(h->P.bvc + d.bvc_off, 0, 2 * su * sizeof(int32_t), st));
    HIPCHK(hipMemsetAsync(h->P.dpart + d.dom_off, 0, job.n_dom * sizeof(DomPart), st));
    HIPCHK(hipMemsetAsync(h->P.sweep + slot, 0, sizeof(unsigned long long), st));
    HIPCHK(hipMemsetAsync(h->P.flags + slot, 0, sizeof(unsigned int), st));
    HIPCHK(hipMemsetAsync(h->P.nnacc + slot, 0, sizeof(unsigned long long), st));
    HIPCHK(hipMemsetAsync(h->P.acc + slot, 0, sizeof(pmwa_obs_acc), st));
    // host view: keep the slot's capacities, take the job's parameters
    hc.p = job.p;
    hc.d = d;
    hc.cdf = job.cdf;
    hc.C = job.C; hc.rho_max = job.rho_max; hc.delta = job.delta;
    hc.n_units_v = job.n_units_v; hc.n_units_r = job.n_units_r; hc.n_dom = job.n_dom;
    hc.n_bt = job.n_bt; hc.n_bsx = job.n_bsx; hc.n_bsy = job.n_bsy;
    hc.enq_sweeps = hc.read_sweeps = 0;
    hc.host_rows.clear();
    hc.active = true;
    hc.target = (uint64_t)target_sweeps;
    return PMWA_OK;
}

int pmwa_slot_release(pmwa_t* h, int slot)
{
    if (!h || !h->slots || slot < 0 || slot >= (int)h->ch.size()) return PMWA_EINVAL;
    HostChain& hc = h->ch[slot];
    HIPCHK(hipEventSynchronize(hc.staged));
    hc.d.active = 0;
    std::memcpy(hc.staging, &hc.d, sizeof(ChainDev));
    HIPCHK(hipMemcpyAsync(h->d_cd + slot, hc.staging, sizeof(ChainDev), hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipEventRecord(hc.staged, h->stream));
    hc.active = false;
    hc.host_rows.clear();
    hc.read_sweeps = hc.enq_sweeps;
    return PMWA_OK;
}

int pmwa_slot_progress(pmwa_t* h, int slot, int64_t* sweeps_done)
{
    if (!h || !sweeps_done || slot < 0 || slot >= (int)h->ch.size()) return PMWA_EINVAL;
    HIPCHK(hipStreamSynchronize(h->stream));
    unsigned long long sw = 0;
    HIPCHK(hipMemcpy(&sw, h->P.sweep + slot, sizeof(sw), hipMemcpyDeviceToHost));
    *sweeps_done = (int64_t)sw;
    return PMWA_OK;
}

int pmwa_phase(pmwa_t* h, int phase)
{
    if (!h || phase < 1 || phase > 7) return PMWA_EINVAL;
    if (phase == 7) {
        for (auto& hc : h->ch)
            if (hc.enq_sweeps - hc.read_sweeps >= (uint64_t)h->opts.series_cap) {
                int rc = drain(h);
                if (rc) return rc;
                break;
            }
    }
    int rc = launch_phases(h, phase, phase);
    if (rc == PMWA_OK && phase == 7) advance_enq(h);
    return rc;
}

static int build_graph(pmwa_t* h)
{
    hipStream_t s = h->stream;
    HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    int rc = PMWA_OK;
    rc = launch_phases(h, 1, 7);
    hipGraph_t g = nullptr;
    if (hipStreamEndCapture(s, &g) != hipSuccess || rc) {
        if (g) (void)hipGraphDestroy(g);
        return PMWA_EDEVICE;
    }
    h->graph = g;
    HIPCHK(hipGraphInstantiate(&h->gexec, g, nullptr, nullptr, 0));
    return PMWA_OK;
}

int pmwa_sweep(pmwa_t* h, int64_t n)
{
    if (!h || n < 0) return PMWA_EINVAL;
    const bool graph = h->opts.use_graph != 0 && !h->timing;
    if (graph && !h->gexec) {
        int rc = build_graph(h);
        if (rc) return rc;
    }
    for (int64_t i = 0; i < n; i++) {
        for (auto& hc : h->ch)
            if (hc.enq_sweeps - hc.read_sweeps >= (uint64_t)h->opts.series_cap) {
                int rc = drain(h);
                if (rc) return rc;
                break;
            }
        if (graph) {
            HIPCHK(hipGraphLaunch(h->gexec, h->stream));
        } else {
            int rc = launch_phases(h, 1, 7);
            if (rc) return rc;
        }
        advance_enq(h);
    }
    return PMWA_OK;
}

int pmwa_status(pmwa_t* h)
{
    if (!h) return PMWA_EINVAL;
    std::vector<unsigned int> f;
    int rc = read_flags(h, f);
    if (rc) return rc;
    for (unsigned int x : f)
        if (x) return flag_code(x);
    return PMWA_OK;
}

int pmwa_measure(pmwa_t* h, int chain, pmwa_obs* out, int64_t max_rows, int64_t* n_rows)
{
    if (!h || chain < 0 || chain >= (int)h->ch.size() || !n_rows || max_rows < 0 || (!out && max_rows)) return PMWA_EINVAL;
    int rc = drain(h);
    if (rc) return rc;
    HostChain& hc = h->ch[chain];
    const int64_t n = std::min<int64_t>(max_rows, (int64_t)hc.host_rows.size());
    if (n > 0) std::memcpy(out, hc.host_rows.data(), n * sizeof(pmwa_obs));
    hc.host_rows.erase(hc.host_rows.begin(), hc.host_rows.begin() + n);
    *n_rows = n;
    std::vector<unsigned int> f;
    rc = read_flags(h, f);
    if (rc) return rc;
    return flag_code(f[chain]);
}

int pmwa_set_timing(pmwa_t* h, int enable)
{
    if (!h) return PMWA_EINVAL;
    h->timing = enable != 0;
    h->timing_mask = enable != 0 ? 0x7Fu : 0u;
    return PMWA_OK;
}

int pmwa_set_timing_phases(pmwa_t* h, uint32_t mask)
{
    if (!h || (mask & ~0x7Fu)) return PMWA_EINVAL;
    h->timing = mask != 0;
    h->timing_mask = mask;
    return PMWA_OK;
}

int pmwa_phase_times(pmwa_t* h, double* ms, int64_t* launches)
{
    if (!h || !ms || !launches) return PMWA_EINVAL;
    HIPCHK(hipStreamSynchronize(h->stream));
    for (int i = 0; i < 7; i++) { ms[i] = 0.0; launches[i] = 0; }
    for (size_t i = 0; i + 1 < h->ev_used; i += 2) {
        float t = 0.0f;
        HIPCHK(hipEventElapsedTime(&t, h->ev_pool[i], h->ev_pool[i + 1]));
        const int ph = h->ev_phase[i / 2];
        ms[ph - 1] += t;
        launches[ph - 1] += 1;
    }
    h->ev_used = 0;
    return PMWA_OK;
}

int pmwa_diag(pmwa_t* h, int chain, int64_t* out, int n)
{
    if (!h || !out || n < 4 || chain < 0 || chain >= (int)h->ch.size()) return PMWA_EINVAL;
    HIPCHK(hipStreamSynchronize(h->stream));
    const HostChain& hc = h->ch[chain];
    std::vector<DomPart> dp(hc.n_dom);
    HIPCHK(hipMemcpy(dp.data(), h->P.dpart + hc.d.dom_off, dp.size() * sizeof(DomPart), hipMemcpyDeviceToHost));
    int64_t wsum = 0, wmax = 0, att = 0, amax = 0;
    for (const DomPart& x : dp) {
        wsum += x.windows;
        wmax = std::max<int64_t>(wmax, x.windows);
        att += x.nw * (int64_t)hc.d.ncycle;
        amax = std::max<int64_t>(amax, x.nw * (int64_t)hc.d.ncycle);
    }
    out[0] = wsum; out[1] = wmax; out[2] = att; out[3] = amax;
    return PMWA_OK;
}

int pmwa_green(pmwa_t* h, int chain, const int32_t* disp, int n, double* out)
{
    if (!h || chain < 0 || chain >= (int)h->ch.size() || n < 1 || n > PMWA_GREEN_MAX || !disp || !out)
        return PMWA_EINVAL;
    const ChainDev& d = h->ch[chain].d;
    HIPCHK(hipStreamSynchronize(h->stream));
    unsigned int fl = 0;
    HIPCHK(hipMemcpy(&fl, h->P.flags + chain, sizeof(fl), hipMemcpyDeviceToHost));
    if (fl) return (fl & 1u) ? PMWA_EOVERFLOW : PMWA_ESTATE;
    // displacements modulo the lattice and beta; (0, 0, 0) gives 1 without a
    // launch
    std::vector<int4> dv;
    std::vector<int> slot(n, -1);
    for (int q = 0; q < n; q++) {
        const int rx = ((disp[3 * q] % d.Lx) + d.Lx) % d.Lx, ry = ((disp[3 * q + 1] % d.Ly) + d.Ly) % d.Ly;
        const int dt = (int)((((int64_t)disp[3 * q + 2] % d.M) + d.M) % d.M);
        if (rx == 0 && ry == 0 && dt == 0) continue;
        slot[q] = (int)dv.size();
        dv.push_back(make_int4(rx, ry, dt, 0));
    }
    std::vector<double> part;
    const int nd = (int)dv.size();
    const int nchunk = (d.N + 63) / 64;
    const size_t nblk = (size_t)d.ntau * nd * nchunk;
    if (nd > 0) {
        if (!h->d_gdisp && hipMalloc(&h->d_gdisp, PMWA_GREEN_MAX * sizeof(int4)) != hipSuccess) {
            h->d_gdisp = nullptr;
            return PMWA_ENOMEM;
        }
        if (nblk > h->gpart_cap) {
            if (h->d_gpart) (void)hipFree(h->d_gpart);
            h->d_gpart = nullptr;
            h->gpart_cap = 0;
            if (hipMalloc(&h->d_gpart, nblk * sizeof(double)) != hipSuccess) return PMWA_ENOMEM;
            h->gpart_cap = nblk;
        }
        HIPCHK(hipMemcpyAsync(h->d_gdisp, dv.data(), nd * sizeof(int4), hipMemcpyHostToDevice, h->stream));
        hipLaunchKernelGGL(k_green, dim3((unsigned)nblk), dim3(64), 0, h->stream, h->P, chain, h->d_gdisp, nd, nchunk,
                           h->d_gpart);
        HIPCHK(hipGetLastError());
        part.resize(nblk);
        HIPCHK(hipMemcpyAsync(part.data(), h->d_gpart, nblk * sizeof(double), hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
    }
    // fixed summation order: slab, then block of sites
    const double norm = (double)d.M * (double)d.N;
    for (int q = 0; q < n; q++) {
        if (slot[q] < 0) { out[q] = 1.0; continue; }
        double sum = 0.0;
        for (int k = 0; k < d.ntau; k++)
            for (int c = 0; c < nchunk; c++) sum += part[((size_t)k * nd + slot[q]) * nchunk + c];
        out[q] = sum / norm;
    }
    return PMWA_OK;
}

int pmwa_chain_status(pmwa_t* h, int chain)
{
    if (!h || chain < 0 || chain >= (int)h->ch.size()) return PMWA_EINVAL;
    HIPCHK(hipStreamSynchronize(h->stream));
    unsigned int fl = 0;
    HIPCHK(hipMemcpy(&fl, h->P.flags + chain, sizeof(fl), hipMemcpyDeviceToHost));
    return flag_code(fl);
}

// standard error of the mean of S samples from their sum and sum of squares
static double sem(double sum, double sq, double S)
{
    if (!(S > 1.0)) return NAN;
    const double m = sum / S;
    const double var = sq / S - m * m;
    return std::sqrt((var > 0.0 ? var : 0.0) / (S - 1.0));
}

int pmwa_observables(pmwa_t* h, int chain, pmwa_summary* out)
{
    if (!h || !out || chain < 0 || chain >= (int)h->ch.size()) return PMWA_EINVAL;
    HIPCHK(hipStreamSynchronize(h->stream));
    const HostChain& hc = h->ch[chain];
    pmwa_obs_acc a;
    HIPCHK(hipMemcpy(&a, h->P.acc + chain, sizeof(a), hipMemcpyDeviceToHost));
    unsigned int fl = 0;
    HIPCHK(hipMemcpy(&fl, h->P.flags + chain, sizeof(fl), hipMemcpyDeviceToHost));
    std::memset(out, 0, sizeof(*out));
    out->acc = a;
    // the estimators, in this operation order
    const double S = (double)a.sweeps, N = (double)hc.d.N, M = (double)hc.d.M;
    const double beta = hc.p.beta, eta = hc.p.eta, V = hc.p.V, mu = hc.p.mu, C = hc.C;
    const double m_nv = (double)a.nv / S, m_nk = (double)a.nkink / S, m_nw = (double)a.nw / S;
    const double m_occ = (double)a.occ2 / S, m_nn = (double)a.nn2 / S, m_q = a.qimp / S;
    out->E = 2.0 * C - m_nv / (beta * N);
    out->E_alt = (V * m_nn - mu * m_occ) / (2.0 * M * N) - m_nk / (beta * N);
    out->E_eta = out->E - m_nw / (beta * N);
    out->density = m_occ / (2.0 * M * N);
    out->Q = m_nw / (beta * eta * N);
    out->Q_imp = m_q / (M * N);
    out->b = 0.5 * out->Q_imp;
    out->err_E = sem((double)a.nv, a.nv_sq, S) / (beta * N);
    out->err_density = sem((double)a.occ2, a.occ2_sq, S) / (2.0 * M * N);
    out->err_Q = sem((double)a.nw, a.nw_sq, S) / (beta * eta * N);
    out->err_Q_imp = sem(a.qimp, a.qimp_sq, S) / (M * N);
    return flag_code(fl);
}

int pmwa_reset_observables(pmwa_t* h)
{
    if (!h) return PMWA_EINVAL;
    const int n = (int)h->ch.size();
    hipLaunchKernelGGL(k_reset_acc, dim3((unsigned)std::min((n + 63) / 64, 1024)), dim3(64), 0, h->stream, h->P, n);
    return hipGetLastError() == hipSuccess ? PMWA_OK : PMWA_EDEVICE;
}

int pmwa_state_hash(pmwa_t* h, int chain, uint64_t* out)
{
    if (!h || !out || chain < 0 || chain >= (int)h->ch.size()) return PMWA_EINVAL;
    const ChainDev& d = h->ch[chain].d;
    const long long units = (long long)d.ntau * d.N;
    HIPCHK(hipMemsetAsync(h->d_hash, 0, sizeof(unsigned long long), h->stream));
    hipLaunchKernelGGL(k_hash, dim3((unsigned)((units + 63) / 64)), dim3(64), 0, h->stream, h->P, chain, h->d_hash);
    HIPCHK(hipGetLastError());
    unsigned long long v = 0;
    HIPCHK(hipMemcpyAsync(&v, h->d_hash, sizeof(v), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    *out = (uint64_t)v;
    return PMWA_OK;
}

int pmwa_correlator(pmwa_t* h, int chain, int npt, const int32_t* pts, int ncorr, int nbase, double* out)
{
    if (!h || chain < 0 || chain >= (int)h->ch.size() || npt < 1 || npt > PMWA_CORR_MAX_POINTS || ncorr < 1 ||
        ncorr > PMWA_CORR_MAX || nbase < 1 || nbase > (1 << 20) || !pts || !out)
        return PMWA_EINVAL;
    const ChainDev& d = h->ch[chain].d;
    std::vector<int4> pv((size_t)ncorr * npt);
    for (int q = 0; q < ncorr * npt; q++) {
        const int32_t* r = pts + 4 * (size_t)q;
        if (r[3] < 0 || r[3] > 2) return PMWA_EINVAL;
        pv[q] = make_int4(((r[0] % d.Lx) + d.Lx) % d.Lx, ((r[1] % d.Ly) + d.Ly) % d.Ly,
                          (int)((((int64_t)r[2] % d.M) + d.M) % d.M), r[3]);
    }
    HIPCHK(hipStreamSynchronize(h->stream));
    unsigned int fl = 0;
    HIPCHK(hipMemcpy(&fl, h->P.flags + chain, sizeof(fl), hipMemcpyDeviceToHost));
    if (fl) return (fl & 1u) ? PMWA_EOVERFLOW : PMWA_ESTATE;
    const long long pairs = (long long)d.N * nbase;
    const long long nchunk = (pairs + 63) / 64;
    const long long nblk = nchunk * ncorr;
    if (nblk > 0x7FFFFFFFLL) return PMWA_EINVAL;
    if (!h->d_cpts &&
        hipMalloc(&h->d_cpts, (size_t)PMWA_CORR_MAX * PMWA_CORR_MAX_POINTS * sizeof(int4)) != hipSuccess) {
        h->d_cpts = nullptr;
        return PMWA_ENOMEM;
    }
    if ((size_t)nblk > h->gpart_cap) {
        if (h->d_gpart) (void)hipFree(h->d_gpart);
        h->d_gpart = nullptr;
        h->gpart_cap = 0;
        if (hipMalloc(&h->d_gpart, (size_t)nblk * sizeof(double)) != hipSuccess) return PMWA_ENOMEM;
        h->gpart_cap = (size_t)nblk;
    }
    HIPCHK(hipMemcpyAsync(h->d_cpts, pv.data(), pv.size() * sizeof(int4), hipMemcpyHostToDevice, h->stream));
    hipLaunchKernelGGL(k_corr, dim3((unsigned)nblk), dim3(64), 0, h->stream, h->P, chain, h->d_cpts, npt, nbase,
                       (int)nchunk, h->d_gpart);
    HIPCHK(hipGetLastError());
    std::vector<double> part((size_t)nblk);
    HIPCHK(hipMemcpyAsync(part.data(), h->d_gpart, nblk * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    const double norm = (double)d.N * (double)nbase;
    for (int c = 0; c < ncorr; c++) {
        double sum = 0.0;
        for (long long b = 0; b < nchunk; b++) sum += part[(size_t)c * nchunk + b];
        out[c] = sum / norm;
    }
    return PMWA_OK;
}

int pmwa_green_static(pmwa_t* h, int chain, const int32_t* disp, int n, double* out)
{
    if (!h || chain < 0 || chain >= (int)h->ch.size() || n < 1 || n > PMWA_GREEN_MAX || !disp || !out)
        return PMWA_EINVAL;
    if (!h->scratch) return PMWA_EDEVICE;
    const ChainDev& d = h->ch[chain].d;
    // the partials of one call must fit the static scratch
    int4 dv[PMWA_GREEN_MAX];
    int slot[PMWA_GREEN_MAX];
    int nd = 0;
    for (int q = 0; q < n; q++) {
        const int rx = ((disp[3 * q] % d.Lx) + d.Lx) % d.Lx, ry = ((disp[3 * q + 1] % d.Ly) + d.Ly) % d.Ly;
        const int dt = (int)((((int64_t)disp[3 * q + 2] % d.M) + d.M) % d.M);
        slot[q] = -1;
        if (rx == 0 && ry == 0 && dt == 0) continue;
        slot[q] = nd;
        dv[nd++] = make_int4(rx, ry, dt, 0);
    }
    const int nchunk = (d.N + 63) / 64;
    const long long nblk = (long long)d.ntau * nd * nchunk;
    if (nblk > PMWA_GREEN_STATIC_PARTIALS) return PMWA_EINVAL;
    HIPCHK(hipStreamSynchronize(h->stream));
    unsigned int fl = 0;
    HIPCHK(hipMemcpy(&fl, h->P.flags + chain, sizeof(fl), hipMemcpyDeviceToHost));
    if (fl) return (fl & 1u) ? PMWA_EOVERFLOW : PMWA_ESTATE;
    double res[PMWA_GREEN_MAX];
    if (nd > 0) {
        unsigned char* base = static_cast<unsigned char*>(h->scratch);
        int4* s_disp = reinterpret_cast<int4*>(base + SCR_DISP);
        double* s_out = reinterpret_cast<double*>(base + SCR_OUT);
        double* s_part = reinterpret_cast<double*>(base + SCR_PART);
        HIPCHK(hipMemcpyAsync(s_disp, dv, nd * sizeof(int4), hipMemcpyHostToDevice, h->stream));
        hipLaunchKernelGGL(k_green, dim3((unsigned)nblk), dim3(64), 0, h->stream, h->P, chain, s_disp, nd, nchunk,
                           s_part);
        HIPCHK(hipGetLastError());
        hipLaunchKernelGGL(k_green_sum, dim3((unsigned)((nd + 63) / 64)), dim3(64), 0, h->stream, s_part, d.ntau,
                           nd, nchunk, (double)d.M * (double)d.N, s_out);
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(res, s_out, nd * sizeof(double), hipMemcpyDeviceToHost, h->stream));
        HIPCHK(hipStreamSynchronize(h->stream));
    }
    for (int q = 0; q < n; q++) out[q] = slot[q] < 0 ? 1.0 : res[slot[q]];
    return PMWA_OK;
}

int pmwa_chain_info(pmwa_t* h, int chain, pmwa_info* out)
{
    if (!h || !out || chain < 0 || chain >= (int)h->ch.size()) return PMWA_EINVAL;
    const HostChain& hc = h->ch[chain];
    out->C = hc.C;
    out->rho_max = hc.rho_max;
    out->delta = hc.delta;
    out->lambda = hc.d.lambda;
    out->n_cycle = hc.d.ncycle;
    out->M = hc.d.M;
    out->event_cap = hc.d.cap;
    out->bond_cap = hc.d.capb;
    out->n_domains = hc.n_dom;
    return PMWA_OK;
}

// canonical layout <-> device layout
int pmwa_get_state(pmwa_t* h, int chain, uint8_t* bstate, int32_t* counts, int32_t* ticks,
                   uint32_t* infos, int64_t cap, int64_t* n_events, uint64_t* sweep)
{
    if (!h || chain < 0 || chain >= (int)h->ch.size() || !n_events) return PMWA_EINVAL;
    HIPCHK(hipStreamSynchronize(h->stream));
    const ChainDev& d = h->ch[chain].d;
    const int64_t su = (int64_t)d.ntau * d.N;
    std::vector<int32_t> cnt(su);
    std::vector<uint8_t> bs(su);
    std::vector<uint2> ev((size_t)su * d.cap);
    HIPCHK(hipMemcpy(cnt.data(), h->P.cnt + d.cnt_off, su * sizeof(int32_t), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(bs.data(), h->P.bs + d.bs_off, su, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(ev.data(), h->P.ev + d.ev_off, ev.size() * sizeof(uint2), hipMemcpyDeviceToHost));
    unsigned long long sw = 0;
    HIPCHK(hipMemcpy(&sw, h->P.sweep + chain, sizeof(sw), hipMemcpyDeviceToHost));
    int64_t total = 0;
    for (int64_t i = 0; i < su; i++) total += cnt[i];
    *n_events = total;
    if (sweep) *sweep = sw;
    if (cap == 0) return PMWA_OK;
    if (cap < total || !bstate || !counts || !ticks || !infos) return PMWA_EINVAL;
    int64_t o = 0;
    for (int k = 0; k < d.ntau; k++)
        for (int site = 0; site < d.N; site++) {
            const int x = site % d.Lx, y = site / d.Lx;
            const int dsp = (y / d.ey) * d.dom_x + x / d.ex, sl = (y % d.ey) * d.ex + x % d.ex;
            const int64_t u = (int64_t)(k * d.ndsp + dsp) * d.nloc + sl;
            bstate[(int64_t)k * d.N + site] = bs[u];
            counts[(int64_t)k * d.N + site] = cnt[u];
            for (int j = 0; j < cnt[u]; j++) {
                const uint2 e = ev[((int64_t)(k * d.ndsp + dsp) * d.cap + j) * d.nloc + sl];
                ticks[o] = (int32_t)e.x;
                infos[o] = e.y;
                o++;
            }
        }
    return PMWA_OK;
}

int pmwa_set_state(pmwa_t* h, int chain, const uint8_t* bstate, const int32_t* counts,
                   const int32_t* ticks, const uint32_t* infos, int64_t n_events, uint64_t sweep)
{
    if (!h || chain < 0 || chain >= (int)h->ch.size() || !bstate || !counts || n_events < 0) return PMWA_EINVAL;
    if (n_events > 0 && (!ticks || !infos)) return PMWA_EINVAL;
    HIPCHK(hipStreamSynchronize(h->stream));
    const ChainDev& d = h->ch[chain].d;
    const int64_t su = (int64_t)d.ntau * d.N;
    std::vector<int32_t> cnt(su);
    std::vector<uint8_t> bs(su);
    std::vector<uint2> ev((size_t)su * d.cap, make_uint2(0, 0));
    int64_t o = 0;
    for (int k = 0; k < d.ntau; k++)
        for (int site = 0; site < d.N; site++) {
            const int x = site % d.Lx, y = site / d.Lx;
            const int dsp = (y / d.ey) * d.dom_x + x / d.ex, sl = (y % d.ey) * d.ex + x % d.ex;
            const int64_t u = (int64_t)(k * d.ndsp + dsp) * d.nloc + sl;
            const int n = counts[(int64_t)k * d.N + site];
            if (n < 0 || n > d.cap || o + n > n_events) return n > d.cap ? PMWA_EOVERFLOW : PMWA_EINVAL;
            if (bstate[(int64_t)k * d.N + site] > 1) return PMWA_ESTATE;
            bs[u] = bstate[(int64_t)k * d.N + site];
            cnt[u] = n;
            int64_t prevkey = -1;
            for (int j = 0; j < n; j++, o++) {
                const int32_t tk = ticks[o];
                const uint32_t inf = infos[o];
                if (tk < d.T[k] || tk >= d.T[k + 1] || (inf & ~15u) || ((inf & 1u) && (inf & 4u))) return PMWA_ESTATE;
                const int64_t key = 2LL * tk + (inf & 1u);
                if (key < prevkey) return PMWA_ESTATE;
                prevkey = key;
                ev[((int64_t)(k * d.ndsp + dsp) * d.cap + j) * d.nloc + sl] = make_uint2((uint32_t)tk, inf);
            }
        }
    if (o != n_events) return PMWA_EINVAL;
    HIPCHK(hipMemcpy(h->P.cnt + d.cnt_off, cnt.data(), su * sizeof(int32_t), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(h->P.bs + d.bs_off, bs.data(), su, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(h->P.ev + d.ev_off, ev.data(), ev.size() * sizeof(uint2), hipMemcpyHostToDevice));
    const unsigned long long sw = sweep;
    HIPCHK(hipMemcpy(h->P.sweep + chain, &sw, sizeof(sw), hipMemcpyHostToDevice));
    const unsigned long long z = 0;
    HIPCHK(hipMemcpy(h->P.nnacc + chain, &z, sizeof(z), hipMemcpyHostToDevice));
    const pmwa_obs_acc za{};
    HIPCHK(hipMemcpy(h->P.acc + chain, &za, sizeof(za), hipMemcpyHostToDevice));
    HostChain& hc = h->ch[chain];
    hc.enq_sweeps = hc.read_sweeps = sweep;
    hc.host_rows.clear();
    return PMWA_OK;
}

}  // extern "C"
